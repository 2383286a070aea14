"""Seeded sweep of ragged shapes through the GPU path against the oracle: the all-at-once matvec
at every FFT length (L = 16 .. 8192, odd and even level counts), P^-1 with the exact shifted
solves at random M and N_t (powers of two and Bluestein lengths), the 1D tau preconditioner at
M = 2^k - 1, and the 2D matvec and tau preconditioner on random grids.  Shapes are drawn once
from a fixed seed, so the sweep is the same on every run."""
import numpy as np
import pytest

from gpu_util import TOL_FFT, TOL_SOLVE, banner, rel_max, to_dev, to_host
from oracle import allatonce as aa
from oracle import precond as pc
from oracle import twod
from rfde_workloads import random_vector

pytestmark = pytest.mark.gpu

_rng = np.random.default_rng(20261203)
MV = [(round(float(_rng.uniform(1.05, 2.0)), 3), int(m), int(_rng.integers(2, 10)))
      for m in np.unique(np.concatenate([_rng.integers(1, 4097, 10),
                                         [1, 8, 9, 64, 65, 129, 1000, 2048, 2049, 4096]]))]
PINV = [(round(float(_rng.uniform(1.05, 2.0)), 3), int(_rng.integers(1, 400)),
         int(_rng.choice([2, 3, 5, 8, 12, 16, 17, 31, 32, 40])))
        for _ in range(8)]
TAU = [(round(float(_rng.uniform(1.05, 2.0)), 3), 2 ** int(k) - 1, int(_rng.integers(2, 40)))
       for k in (3, 5, 7, 8, 9, 10, 11, 12)]
GRID = [(round(float(_rng.uniform(1.1, 1.9)), 3), round(float(_rng.uniform(1.1, 1.9)), 3),
         2 ** int(kx) - 1, 2 ** int(ky) - 1, int(_rng.integers(2, 12)))
        for kx, ky in ((2, 6), (6, 2), (4, 5), (7, 3), (5, 7))]
# the shortest DST-I lengths (M = 1 and 3: transforms of length 4 and 8); the fewest rows of
# the half-length kernel (N_t = 2: rows 0 and 1 packed into one item; N_t = 3: two items, none
# packed) at every rows-per-workgroup count (M = 4095 .. 255), and an odd N_t at M = 4095
TAU += [(1.5, 1, 4), (1.9, 3, 7)]
TAU += [(1.7, 4095, 2), (1.3, 4095, 3), (1.6, 2047, 2), (1.4, 1023, 3), (1.8, 511, 2),
        (1.2, 255, 3), (1.5, 4095, 31)]
GRID += [(1.3, 1.7, 1, 7, 4), (1.6, 1.2, 3, 3, 5), (1.8, 1.1, 1, 1, 3)]


def _plan(alpha, M, Nt, **kw):
    from paper_2003_07020_amd.rfde import Plan
    return Plan.create_1d(alpha, 1.0, 0.0, 1.0, M, Nt, 1.0, **kw)


@pytest.mark.parametrize("alpha,M,Nt", MV)
def test_matvec_sweep(alpha, M, Nt):
    banner(f"sweep matvec alpha={alpha} M={M} Nt={Nt}")
    p = _plan(alpha, M, Nt)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    A = aa.jacobian_A(alpha, 1.0, h, M)
    v = random_vector(M + Nt, Nt * M).reshape(Nt, M)
    y = to_host(p.apply_A(to_dev(v.ravel()))).reshape(Nt, M)
    assert rel_max(y, aa.apply_all_at_once(v, A, tau)) < TOL_FFT


@pytest.mark.parametrize("alpha,M,Nt", PINV)
def test_pinv_exact_sweep(alpha, M, Nt):
    banner(f"sweep pinv alpha={alpha} M={M} Nt={Nt}")
    p = _plan(alpha, M, Nt)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    A = aa.jacobian_A(alpha, 1.0, h, M)
    v = random_vector(3 * M + Nt, Nt * M).reshape(Nt, M)
    z = to_host(p.apply_Pinv(to_dev(v.ravel()))).reshape(Nt, M)
    # rounding of the shifted solves (u cond(B_n), cond up to ~(M+1)^alpha) amplified by the
    # 1/s_j >= 1/eps = 2 N_t of step (c)
    eps = pc.default_eps(tau)
    tol = max(TOL_SOLVE, 1e-15 * (M + 1) ** alpha / eps)
    assert rel_max(z, pc.pinv_fast(v, A, tau, eps)) < tol


@pytest.mark.parametrize("alpha,M,Nt", TAU)
def test_pinv_tau_sweep(alpha, M, Nt):
    from paper_2003_07020_amd import _lib as capi
    banner(f"sweep tau alpha={alpha} M={M} Nt={Nt}")
    p = _plan(alpha, M, Nt, spatial="tau")
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    # the plan's own sigma (eq. (3.10) cancels for the smallest eigenvalues; its rounding is
    # checked separately against the bound of that sum)
    sig_A = -(1.0 / h**alpha) * to_host(p.export(capi.EXPORT_TAU_SIGMA))
    v = random_vector(5 * M + Nt, Nt * M).reshape(Nt, M)
    z = to_host(p.apply_Pinv(to_dev(v.ravel()))).reshape(Nt, M)
    assert rel_max(z, pc.pinv_tau(v, sig_A, tau, pc.default_eps(tau))) < TOL_SOLVE


@pytest.mark.parametrize("gx,gy,Mx,My,Nt", GRID)
def test_2d_sweep(gx, gy, Mx, My, Nt):
    from paper_2003_07020_amd.rfde import Plan
    banner(f"sweep 2d {gx},{gy} {Mx}x{My} Nt={Nt}")
    p = Plan.create_2d(gx, gy, 1.0, 1.0, 0.0, 1.0, 0.0, 1.0, Mx, My, Nt, 1.0)
    hx, hy, tau = 1.0 / (Mx + 1), 1.0 / (My + 1), 1.0 / Nt
    Tx, Ty = aa.toeplitz_T(gx, Mx), aa.toeplitz_T(gy, My)
    cx, cy = twod.coeffs(gx, gy, 1.0, 1.0, hx, hy)
    v = random_vector(Mx * My + Nt, Nt * My * Mx).reshape(Nt, My, Mx)
    y = to_host(p.apply_A(to_dev(v.ravel()))).reshape(Nt, My, Mx)
    assert rel_max(y, twod.apply_all_at_once_2d(v, Tx, Ty, cx, cy, tau)) < TOL_FFT
    sx, sy = twod.tau_sigma_2d(gx, gy, Mx, My)
    z = to_host(p.apply_Pinv(to_dev(v.ravel()))).reshape(Nt, My, Mx)
    ref = twod.pinv_tau_2d(v, sx, sy, cx, cy, tau, pc.default_eps(tau))
    assert rel_max(z, ref) < TOL_SOLVE
