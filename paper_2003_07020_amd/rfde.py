"""Python face of the rfde C ABI: torch tensors carry device memory and streams; every step of
the solver runs in the HIP library (librfde.so).  No computation happens here."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t: torch.Tensor, dtype, numel: int, name: str):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")


def opts(tol=1e-8, maxit=200, restart=30, circ_eps=0.0, precond_bits=64, spatial="exact",
         inner_iters=0, inner_tol=0.0) -> L.Opts:
    o = L.Opts()
    L.lib().rfde_opts_default(C.byref(o))
    o.tol, o.maxit, o.restart, o.circ_eps = tol, maxit, restart, circ_eps
    o.precond_bits = precond_bits
    o.spatial = {"exact": L.SPATIAL_EXACT, "tau": L.SPATIAL_TAU,
                 "toeplitz": L.SPATIAL_TOEPLITZ}[spatial]
    o.inner_iters, o.inner_tol = inner_iters, inner_tol
    return o


def release_cached_memory() -> int:
    """Return the library's cached device blocks to the HIP runtime; bytes released."""
    return int(L.lib().rfde_release_cached_memory())


def gk(alpha: float, n: int) -> torch.Tensor:
    """g_0..g_{n-1} computed on the device."""
    g = torch.empty(n, dtype=torch.float64, device="cuda")
    L.check(L.lib().rfde_gk(alpha, n, _ptr(g), _stream()), "rfde_gk")
    return g


def probe_mfma(kind: int, iters: int = 4096) -> float:
    """Sustained matrix-core TFLOP/s of one instruction form (rfde_probe_mfma): kind 0 FP64
    16x16x4, 1 FP32 16x16x4, 2 BF16 16x16x16, 3 BF16 16x16x32."""
    out = C.c_double(0.0)
    L.check(L.lib().rfde_probe_mfma(kind, iters, C.byref(out), _stream()), "rfde_probe_mfma")
    return out.value


@dataclass
class SolveStats:
    """Per-solve statistics (rfde_stats).  ms_pinv_est / ms_matvec_est are estimates: the first
    application's time (HIP events) times n_pinv / n_matvec; ms_solve is wall time."""
    iters: int
    restarts: int
    converged: bool
    true_rel_res: float
    ms_setup: float
    ms_solve: float
    n_pinv: int
    n_matvec: int
    ms_pinv_est: float
    ms_matvec_est: float
    res_hist: list

    @classmethod
    def from_c(cls, st):
        return cls(st.iters, st.restarts, bool(st.converged), st.true_rel_res, st.ms_setup,
                   st.ms_solve, st.n_pinv, st.n_matvec, st.ms_pinv_est, st.ms_matvec_est,
                   [st.res_hist[k] for k in range(st.n_hist)])


class Plan:
    """An rfde plan (1D or 2D).  Use Plan.create_1d / Plan.create_2d."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle
        info = L.PlanInfo()
        L.check(L.lib().rfde_plan_get_info(self._h, C.byref(info)), "rfde_plan_get_info")
        self.info = {k: getattr(info, k) for k, _ in L.PlanInfo._fields_}
        self.dim = info.dim
        self.Nt = info.Nt
        self.nf = info.n_freq
        self.S = info.M if info.dim == 1 else info.Mx * info.My
        self.N = self.Nt * self.S

    @classmethod
    def create_1d(cls, alpha, kappa, a, b, M, Nt, T, **kw):
        h = C.c_void_p()
        o = opts(**kw)
        L.check(L.lib().rfde_plan_create_1d(C.byref(h), alpha, kappa, a, b, M, Nt, T, C.byref(o),
                                            _stream()), "rfde_plan_create_1d")
        return cls(h)

    @classmethod
    def create_2d(cls, alpha_x, alpha_y, kappa_x, kappa_y, ax, bx, ay, by, Mx, My, Nt, T, **kw):
        h = C.c_void_p()
        o = opts(**kw)
        L.check(L.lib().rfde_plan_create_2d(C.byref(h), alpha_x, alpha_y, kappa_x, kappa_y, ax, bx,
                                            ay, by, Mx, My, Nt, T, C.byref(o), _stream()),
                "rfde_plan_create_2d")
        return cls(h)

    def destroy(self):
        if self._h:
            L.lib().rfde_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()

    # ---- individual steps (async on the current stream) ----
    def build_rhs(self, u0: torch.Tensor, f: torch.Tensor, out: torch.Tensor | None = None):
        _need(u0, torch.float64, self.S, "u0")
        _need(f, torch.float64, self.N, "f")
        F = torch.empty_like(f) if out is None else out
        L.check(L.lib().rfde_build_rhs(self._h, _ptr(u0), _ptr(f), _ptr(F)), "rfde_build_rhs")
        return F

    def apply_A(self, v: torch.Tensor, out: torch.Tensor | None = None):
        _need(v, torch.float64, self.N, "v")
        y = torch.empty_like(v) if out is None else out
        L.check(L.lib().rfde_apply_A(self._h, _ptr(v), _ptr(y)), "rfde_apply_A")
        return y

    def step_a(self, v: torch.Tensor):
        _need(v, torch.float64, self.N, "v")
        z1 = torch.empty(self.nf * self.S, dtype=torch.complex128, device=v.device)
        L.check(L.lib().rfde_pinv_step_a(self._h, _ptr(v), _ptr(z1)), "rfde_pinv_step_a")
        return z1

    def step_b(self, z1: torch.Tensor, out: torch.Tensor | None = None):
        _need(z1, torch.complex128, self.nf * self.S, "z1")
        z2 = torch.empty_like(z1) if out is None else out
        L.check(L.lib().rfde_pinv_step_b(self._h, _ptr(z1), _ptr(z2)), "rfde_pinv_step_b")
        return z2

    def step_c(self, z2: torch.Tensor):
        _need(z2, torch.complex128, self.nf * self.S, "z2")
        v = torch.empty(self.N, dtype=torch.float64, device=z2.device)
        L.check(L.lib().rfde_pinv_step_c(self._h, _ptr(z2), _ptr(v)), "rfde_pinv_step_c")
        return v

    def apply_Pinv(self, v: torch.Tensor, out: torch.Tensor | None = None):
        _need(v, torch.float64, self.N, "v")
        z = torch.empty_like(v) if out is None else out
        L.check(L.lib().rfde_apply_Pinv(self._h, _ptr(v), _ptr(z)), "rfde_apply_Pinv")
        return z

    def export(self, what: int, index: int = 0) -> torch.Tensor:
        i = self.info
        if what == L.EXPORT_GK:
            t = torch.empty(i["M"] if i["dim"] == 1 else i["Mx"] + i["My"], dtype=torch.float64)
        elif what == L.EXPORT_SYMBOL:
            n = i["L"] // 2 + 1 if i["dim"] == 1 else i["Lx"] // 2 + 1 + i["Ly"] // 2 + 1
            t = torch.empty(n, dtype=torch.float64)
        elif what == L.EXPORT_LAMBDA:
            t = torch.empty(i["n_freq"], dtype=torch.complex128)
        elif what == L.EXPORT_SCALE:
            t = torch.empty(i["Nt"], dtype=torch.float64)
        elif what == L.EXPORT_FACTOR:
            dt = torch.complex64 if i["precond_bits"] == 32 else torch.complex128
            t = torch.empty(i["Mp"] * i["Mp"], dtype=dt)
        elif what == L.EXPORT_TOEPLITZ_X:
            t = torch.empty(i["M"], dtype=torch.complex128)
        elif what == L.EXPORT_TAU_SIGMA:
            t = torch.empty(i["M"] if i["dim"] == 1 else i["Mx"] + i["My"], dtype=torch.float64)
        else:
            raise ValueError(what)
        t = t.cuda()
        L.check(L.lib().rfde_plan_export(self._h, what, index, _ptr(t)), "rfde_plan_export")
        return t

    def autotune(self) -> dict:
        r = L.TuneReport()
        L.check(L.lib().rfde_plan_autotune(self._h, C.byref(r)), "rfde_plan_autotune")
        return {"time_variant": r.time_variant, "matvec_variant": r.matvec_variant,
                "trsv_grid_cap": r.trsv_grid_cap, "from_cache": r.from_cache,
                "ms_time": list(r.ms_time), "ms_matvec": list(r.ms_matvec),
                "trsv_caps": list(r.trsv_caps), "ms_trsv": list(r.ms_trsv)}

    def set_variants(self, time_variant: int = 0, matvec_variant: int = 0, trsv_grid_cap: int = 0):
        L.check(L.lib().rfde_plan_set_variants(self._h, time_variant, matvec_variant,
                                               trsv_grid_cap), "rfde_plan_set_variants")

    def solve(self, u0: torch.Tensor, f: torch.Tensor, U_init: torch.Tensor | None = None,
              tol: float = 0.0, out: torch.Tensor | None = None, allow_notconv: bool = False):
        _need(u0, torch.float64, self.S, "u0")
        _need(f, torch.float64, self.N, "f")
        if U_init is not None:
            _need(U_init, torch.float64, self.N, "U_init")
        U = torch.empty_like(f) if out is None else out
        st = L.Stats()
        allow = (L.RFDE_OK, L.RFDE_ENOTCONV) if allow_notconv else (L.RFDE_OK,)
        rc = L.check(L.lib().rfde_solve(self._h, _ptr(u0), _ptr(f), _ptr(U_init), _ptr(U), tol,
                                        C.byref(st)), "rfde_solve", allow)
        stats = SolveStats.from_c(st)
        return U, stats, rc


class Batch:
    """Many independent 1D problems solved together (rfde_batch_*): instances are dicts or
    tuples (alpha, kappa, a, b, T, M, Nt).  Marshalling only."""

    def __init__(self, instances, mem_budget: int = 0, **kw):
        inst = []
        for x in instances:
            if isinstance(x, dict):
                x = (x["alpha"], x["kappa"], x.get("a", 0.0), x.get("b", 1.0), x.get("T", 1.0),
                     x["M"], x["Nt"])
            inst.append(L.Instance(*[float(v) for v in x[:5]], int(x[5]), int(x[6])))
        self.sizes = [(i.M, i.Nt) for i in inst]
        arr = (L.Instance * len(inst))(*inst)
        o = opts(**kw)
        h = C.c_void_p()
        L.check(L.lib().rfde_batch_create(C.byref(h), len(inst), arr, C.byref(o), int(mem_budget),
                                          _stream()), "rfde_batch_create")
        self._h = h

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.lib().rfde_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    @property
    def info(self) -> dict:
        bi = L.BatchInfo()
        L.check(L.lib().rfde_batch_get_info(self._h, C.byref(bi)), "rfde_batch_get_info")
        return {k: getattr(bi, k) for k, _ in L.BatchInfo._fields_}

    def wave_of(self, index: int) -> int:
        w = L.lib().rfde_batch_wave_of(self._h, index)
        if w < 0:
            raise L.RfdeError(w, "rfde_batch_wave_of")
        return w

    def set_autotune(self, what: int = 3):
        L.check(L.lib().rfde_batch_set_autotune(self._h, what), "rfde_batch_set_autotune")

    def set_grid_caps(self, factor_cap: int = 0, trsv_cap: int = 0):
        L.check(L.lib().rfde_batch_set_grid_caps(self._h, factor_cap, trsv_cap),
                "rfde_batch_set_grid_caps")

    def solve(self, u0s, fs, outs=None, allow_notconv: bool = False):
        n = len(self.sizes)
        if len(u0s) != n or len(fs) != n:
            raise ValueError("one u0 and one f per instance")
        for (M, Nt), u0, f in zip(self.sizes, u0s, fs):
            _need(u0, torch.float64, M, "u0")
            _need(f, torch.float64, M * Nt, "f")
        outs = outs or [torch.empty_like(f) for f in fs]
        P = C.c_void_p * n
        st = (L.Stats * n)()
        allow = (L.RFDE_OK, L.RFDE_ENOTCONV) if allow_notconv else (L.RFDE_OK,)
        rc = L.check(L.lib().rfde_batch_solve(self._h, P(*[t.data_ptr() for t in u0s]),
                                              P(*[t.data_ptr() for t in fs]),
                                              P(*[t.data_ptr() for t in outs]), st),
                     "rfde_batch_solve", allow)
        stats = [SolveStats.from_c(s) for s in st]
        return outs, stats, rc


def solve(alpha: float, kappa: float, domain, M: int, Nt: int, T: float, u0: torch.Tensor,
          f: torch.Tensor, tol: float = 1e-8, U_init: torch.Tensor | None = None, **kw):
    """One-call 1D solve (plan, solve, release): the problem of eq. (1.1) on (a, b) x (0, T]
    with M interior points and Nt BDF2 steps; u0 [M], f [Nt][M] FP64 device tensors (f at
    t_1..t_Nt).  Returns (U [Nt * M], SolveStats)."""
    a, b = domain
    with Plan.create_1d(alpha, kappa, a, b, M, Nt, T, tol=tol, **kw) as p:
        U, st, _ = p.solve(u0, f, U_init=U_init)
    return U, st
