"""Learned initial guess for the all-at-once solve (a growth direction beyond the paper).

The all-at-once solution is linear in the data (eq. (2.11)), so for data
u0 = sum_k a_k sin(k pi x), f = e^{-t} sum_k b_k sin(k pi x) it is sum_j c_j G_j with
c = (a_1..a_8, b_1..b_8) and G_j the solution for the j-th unit data component.  A small MLP
(C ABI rfde_mlp_*; forward, backward and Adam are HIP kernels, the output layer on BF16 MFMAs)
predicts the G_j, in the first Ks sine modes of x, from (alpha, log kappa, log(tau / h^alpha)).
The guess for an instance is assembled on the device and handed to rfde_solve as U_init; the
solver's true FP64 residual decides convergence, and a zero guess is the fallback whenever the
guess's residual is not smaller than ||F||.

Training data are produced by the method itself: for each drawn (alpha, kappa) one plan is
created (by default with the factor-free exact step (b)) and the 16 unit components are solved
(16 FP64 solves per draw), then projected on the
first Ks sine modes (rfde_project_sine).  Targets are scaled by 1/mode^2, the standard deviation
of the synthetic coefficients, so the loss weighs each component by its share in a typical
solution.

This module only marshals arguments and drives the loops; it performs no arithmetic on data.
"""
from __future__ import annotations

import ctypes as C
import math
import time

import numpy as np
import torch

from . import _lib as L
from .rfde import Plan, _ptr, _stream


class MlpStruct(C.Structure):
    _fields_ = [("Pin", C.c_int), ("H1", C.c_int), ("H2", C.c_int), ("NOUT", C.c_int)] + \
        [(n, C.c_void_p) for n in ("W1", "b1", "W2", "b2", "W3t", "b3", "W3t_bf16",
                                   "mW1", "vW1", "mb1", "vb1", "mW2", "vW2", "mb2", "vb2",
                                   "mW3", "vW3", "mb3", "vb3", "mu", "sd")]


def _bind():
    lib = L.lib()
    vp = C.c_void_p
    lib.rfde_mlp_workspace_bytes.argtypes = [C.POINTER(MlpStruct), C.c_int]
    lib.rfde_mlp_workspace_bytes.restype = C.c_size_t
    lib.rfde_mlp_forward.argtypes = [C.POINTER(MlpStruct), vp, C.c_int, vp, vp, vp]
    lib.rfde_mlp_forward_noalloc.argtypes = [C.POINTER(MlpStruct), vp, C.c_int, vp, vp]
    lib.rfde_mlp_forward_noalloc_max_bytes.argtypes = []
    lib.rfde_mlp_forward_noalloc_max_bytes.restype = C.c_size_t
    lib.rfde_mlp_grads.argtypes = [C.POINTER(MlpStruct), vp, vp, C.c_int, vp, vp, vp, vp, vp]
    lib.rfde_mlp_train_step.argtypes = [C.POINTER(MlpStruct), vp, vp, C.c_int, vp, C.c_float,
                                        C.c_int, vp, vp, vp]
    lib.rfde_f32_to_bf16.argtypes = [C.c_size_t, vp, vp, vp]
    lib.rfde_sine_table.argtypes = [C.c_int, C.c_int, vp, vp]
    lib.rfde_guess_assemble.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp]
    lib.rfde_project_sine.argtypes = [C.c_int, C.c_int, C.c_int, vp, vp, C.c_double, vp, vp]
    for n in ("rfde_mlp_forward", "rfde_mlp_forward_noalloc", "rfde_mlp_grads", "rfde_mlp_train_step", "rfde_f32_to_bf16",
              "rfde_sine_table", "rfde_guess_assemble", "rfde_project_sine"):
        getattr(lib, n).restype = C.c_int
    return lib


class GuessNet:
    """Device parameters, Adam state and workspace of the guess network."""

    def __init__(self, Pin, H1, H2, NOUT, mu, sd, seed=0, init_scale=0.05, max_batch=32):
        self.lib = _bind()
        self.Pin, self.H1, self.H2, self.NOUT = Pin, H1, H2, NOUT
        rng = np.random.default_rng(seed)
        host = [rng.standard_normal((H1, Pin)) / math.sqrt(Pin), np.zeros(H1),
                rng.standard_normal((H2, H1)) / math.sqrt(H1), np.zeros(H2),
                rng.standard_normal((NOUT, H2)) * init_scale / math.sqrt(H2), np.zeros(NOUT)]
        self.set_params(host)
        self.mu = torch.tensor(np.asarray(mu, np.float32), device="cuda")
        self.sd = torch.tensor(np.asarray(sd, np.float32), device="cuda")
        self.moments = [torch.zeros_like(p) for p in self.params for _ in range(2)]
        self.max_batch = max_batch
        self._refresh_struct()
        nbytes = self.lib.rfde_mlp_workspace_bytes(C.byref(self.s), max_batch)
        self.ws = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        self.g = torch.empty(max_batch * NOUT, dtype=torch.float32, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.t = 0

    def set_params(self, host_params):
        """Upload parameters (host arrays, order W1, b1, W2, b2, W3t, b3) and derive W3t_bf16."""
        self.params = [torch.tensor(np.asarray(a, np.float32), device="cuda").contiguous()
                       for a in host_params]
        self.W3b = torch.empty(self.params[4].numel(), dtype=torch.int16, device="cuda")
        L.check(_bind().rfde_f32_to_bf16(self.params[4].numel(), _ptr(self.params[4]),
                                         _ptr(self.W3b), _stream()), "rfde_f32_to_bf16")
        if hasattr(self, "s"):
            self._refresh_struct()

    def _refresh_struct(self):
        s = MlpStruct()
        s.Pin, s.H1, s.H2, s.NOUT = self.Pin, self.H1, self.H2, self.NOUT
        names = ("W1", "b1", "W2", "b2", "W3t", "b3")
        for n, p in zip(names, self.params):
            setattr(s, n, p.data_ptr())
        s.W3t_bf16 = self.W3b.data_ptr()
        mom = ("mW1", "vW1", "mb1", "vb1", "mW2", "vW2", "mb2", "vb2", "mW3", "vW3", "mb3", "vb3")
        for n, m in zip(mom, self.moments if hasattr(self, "moments") else [None] * 12):
            setattr(s, n, m.data_ptr() if m is not None else None)
        s.mu = self.mu.data_ptr() if hasattr(self, "mu") else None
        s.sd = self.sd.data_ptr() if hasattr(self, "sd") else None
        self.s = s

    def forward(self, feats: torch.Tensor) -> torch.Tensor:
        B = feats.shape[0]
        self._refresh_struct()
        L.check(self.lib.rfde_mlp_forward(C.byref(self.s), _ptr(feats), B, _ptr(self.g),
                                          _ptr(self.ws), _stream()), "rfde_mlp_forward")
        return self.g[: B * self.NOUT].view(B, self.NOUT)

    def forward_noalloc(self, feats: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """forward() through rfde_mlp_forward_noalloc (no workspace; the library's fixed device
        array holds the activations).  out: float32 device tensor of B * NOUT entries."""
        B = feats.shape[0]
        self._refresh_struct()
        L.check(self.lib.rfde_mlp_forward_noalloc(C.byref(self.s), _ptr(feats), B, _ptr(out),
                                                  _stream()), "rfde_mlp_forward_noalloc")
        return out[: B * self.NOUT].view(B, self.NOUT)

    def grads(self, feats, y):
        B = feats.shape[0]
        self._refresh_struct()
        n = sum(p.numel() for p in self.params)
        out = torch.empty(n, dtype=torch.float32, device="cuda")
        L.check(self.lib.rfde_mlp_grads(C.byref(self.s), _ptr(feats), _ptr(y), B, _ptr(self.g),
                                        _ptr(out), _ptr(self.loss), _ptr(self.ws), _stream()),
                "rfde_mlp_grads")
        parts, o = [], 0
        for p in self.params:
            parts.append(out[o:o + p.numel()].view(p.shape))
            o += p.numel()
        return parts, self.loss

    def train_step(self, feats, y, lr):
        B = feats.shape[0]
        self.t += 1
        self._refresh_struct()
        L.check(self.lib.rfde_mlp_train_step(C.byref(self.s), _ptr(feats), _ptr(y), B,
                                             _ptr(self.g), C.c_float(lr), self.t, _ptr(self.loss),
                                             _ptr(self.ws), _stream()), "rfde_mlp_train_step")
        return self.loss


class LearnedGuess:
    """Training-data generation through the solver, training, and guesses for new instances."""

    def __init__(self, M, Nt, units, T=1.0, Ks=64, H1=64, H2=128, seed=0):
        """units: the 16 unit data components as host arrays (u0[M], f[Nt][M]); component j
        has sine mode (j % 8) + 1."""
        self.M, self.Nt, self.T, self.Ks = M, Nt, T, Ks
        self.nsrc = len(units)
        nmodes = self.nsrc // 2
        self.h, self.tau = 1.0 / (M + 1), T / Nt
        self.NOUT = self.nsrc * Nt * Ks
        # fixed standardisation of (alpha, log kappa, log(tau / h^alpha)) from the parameter laws
        sd_a = 0.8 / math.sqrt(12.0)
        lh = -math.log(self.h)
        mu = [1.5, 0.0, math.log(self.tau) + 1.5 * lh]
        sd = [sd_a, 0.5, sd_a * lh]
        self.net = GuessNet(3, H1, H2, self.NOUT, mu, sd, seed=seed)
        # output scale per unit component: mode^2 (targets are G_j / mode_j^2)
        self.scale = np.array([((j % nmodes) + 1) ** 2 for j in range(self.nsrc)], np.float64)
        self.S = torch.empty(M * Ks, dtype=torch.float64, device="cuda")
        L.check(self.net.lib.rfde_sine_table(M, Ks, _ptr(self.S), _stream()), "rfde_sine_table")
        self.units = [tuple(torch.from_numpy(np.ascontiguousarray(a, np.float64).ravel()).cuda()
                            for a in u) for u in units]

    def features(self, alpha, kappa):
        return [alpha, math.log(kappa), math.log(self.tau / self.h ** alpha)]

    def generate(self, draws, tol=1e-8, spatial="toeplitz", log=None):
        """Targets for a list of (alpha, kappa): 16 FP64 solves per draw, by default with the
        factor-free exact step (b) (the same preconditioner as the LDL^T form, without the
        factorisation: its setup is cheap enough to amortise over 16 solves).  Returns (feats,
        Y) device tensors, Y scaled per component (B x NOUT, float32), and the solve count."""
        n = len(draws)
        Y = torch.empty((n, self.NOUT), dtype=torch.float32, device="cuda")
        feats = torch.tensor([self.features(a, k) for a, k in draws], dtype=torch.float32,
                             device="cuda")
        U = torch.empty(self.Nt * self.M, dtype=torch.float64, device="cuda")
        blk = self.Nt * self.Ks
        solves = 0
        t0 = time.perf_counter()
        for d, (alpha, kappa) in enumerate(draws):
            with Plan.create_1d(alpha, kappa, 0.0, 1.0, self.M, self.Nt, self.T, tol=tol,
                                spatial=spatial) as p:
                for j, (u0, f) in enumerate(self.units):
                    p.solve(u0, f, out=U)
                    solves += 1
                    dst = C.c_void_p(Y.data_ptr() + 4 * (d * self.NOUT + j * blk))
                    L.check(self.net.lib.rfde_project_sine(self.Nt, self.M, self.Ks, _ptr(U),
                                                           _ptr(self.S), 1.0 / self.scale[j],
                                                           dst, _stream()),
                            "rfde_project_sine")
            if log and (d + 1) % max(1, n // 10) == 0:
                log(f"generated {d + 1}/{n} draws ({solves} solves, "
                    f"{time.perf_counter() - t0:.1f} s)")
        return feats, Y, solves

    def train(self, feats, Y, epochs=200, batch=32, lr0=2e-3, lr1=2e-5, seed=1, log=None):
        n = feats.shape[0]
        rng = np.random.default_rng(seed)
        steps_per_epoch = max(1, (n + batch - 1) // batch)
        total = epochs * steps_per_epoch
        it = 0
        hist = []
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(n)).cuda()
            for s0 in range(0, n, batch):
                idx = perm[s0:s0 + batch]
                lr = lr1 + 0.5 * (lr0 - lr1) * (1 + math.cos(math.pi * it / max(1, total - 1)))
                loss = self.net.train_step(feats[idx].contiguous(), Y[idx].contiguous(), lr)
                it += 1
            if (ep + 1) % max(1, epochs // 10) == 0 or ep + 1 == epochs:
                hist.append(float(loss.item()))
                if log:
                    log(f"epoch {ep + 1}/{epochs} loss {hist[-1]:.3e}")
        return hist

    def guess(self, alpha, kappa, coef):
        """Initial guess U_init (device, FP64, [Nt * M]) for data coefficients coef (16)."""
        feats = torch.tensor([self.features(alpha, kappa)], dtype=torch.float32, device="cuda")
        g = self.net.forward(feats)
        cs = torch.tensor(np.asarray(coef, np.float64) * self.scale, device="cuda")
        U = torch.empty(self.Nt * self.M, dtype=torch.float64, device="cuda")
        L.check(self.net.lib.rfde_guess_assemble(self.nsrc, self.Nt, self.Ks, self.M, _ptr(g),
                                                 _ptr(cs), _ptr(self.S), _ptr(U), _stream()),
                "rfde_guess_assemble")
        return U
