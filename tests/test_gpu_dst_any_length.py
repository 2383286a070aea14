"""GPU parity of the tau preconditioner (eq. (3.9)-(3.11), eq. (4.5)) at grid sizes whose DST-I
length n has 2(n+1) not a power of two: the chirp-z DST-I path against the oracle's dense DST
matrix -- step (b), P^-1 and full solves in 1D and 2D (also with one axis of each kind), FP64
and FP32 -- plus a power-of-two case through the same tests, which must stay on the FFT path."""
import numpy as np
import pytest

from gpu_util import banner, rel_max, to_dev, to_host
from oracle import allatonce as aa
from oracle import precond as pc
from oracle import twod
from oracle.weights import gk_recurrence
import rfde_workloads as wl

pytestmark = pytest.mark.gpu


def _plan1d(alpha, M, Nt, **kw):
    from paper_2003_07020_amd.rfde import Plan
    return Plan.create_1d(alpha, 1.0, 0.0, 1.0, M, Nt, 1.0, spatial="tau", **kw)


@pytest.mark.parametrize("alpha,M,Nt", [(1.5, 1, 4), (1.3, 2, 3), (1.7, 5, 8), (1.6, 59, 16),
                                        (1.5, 100, 64), (1.8, 1000, 8), (1.2, 2730, 5),
                                        (1.9, 4000, 4), (1.5, 63, 8)])
@pytest.mark.parametrize("bits", [64, 32])
def test_tau_step_b_any_length_1d(alpha, M, Nt, bits):
    from paper_2003_07020_amd import capi
    banner(f"tau1d any length bits={bits} alpha={alpha} M={M} Nt={Nt}")
    p = _plan1d(alpha, M, Nt, precond_bits=bits)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    eps = pc.default_eps(tau)
    g = gk_recurrence(alpha, M)
    sig_gpu = to_host(p.export(capi.EXPORT_TAU_SIGMA))
    sig_or = pc.tau_eigenvalues(g)
    # rounding bound of the cancelling sine sums of eq. (3.10) (see test_tau_step_b_1d)
    Q = pc.dst_matrix(M)
    bound = (np.abs(Q) @ np.abs(pc.tau_first_column(g))) / np.abs(Q[:, 0])
    u = np.finfo(np.float64).eps / 2
    assert np.all(np.abs(sig_gpu - sig_or) <= (M + 4 * np.log2(2 * (M + 1))) * u * bound)
    sig_A = -(1.0 / h**alpha) * sig_gpu
    v = wl.random_vector(51, Nt * M).reshape(Nt, M)
    z1 = pc.step_a(v, eps)
    z2 = to_host(p.step_b(to_dev(z1.ravel()))).reshape(-1, M)
    # two DSTs by chirp-z: FFTs of length LB ~ 2n plus the chirp products, rounding ~ u log2 LB
    assert rel_max(z2, pc.step_b_tau(z1, sig_A, tau, Nt, eps)) < (1e-11 if bits == 64 else 2e-5)
    z = to_host(p.apply_Pinv(to_dev(v.ravel()))).reshape(Nt, M)
    assert rel_max(z, pc.pinv_tau(v, sig_A, tau, eps)) < (1e-10 if bits == 64 else 1e-4)


@pytest.mark.parametrize("alpha,M,Nt", [(1.5, 100, 64), (1.7, 1000, 128), (1.3, 60, 7)])
@pytest.mark.parametrize("bits", [64, 32])
def test_tau_solve_any_length_1d(alpha, M, Nt, bits):
    banner(f"tau1d solve any length bits={bits} alpha={alpha} M={M} Nt={Nt}")
    p = _plan1d(alpha, M, Nt, precond_bits=bits)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    u0, f, _ = wl.gen1d(52, M, Nt)
    U, st, _ = p.solve(to_dev(u0), to_dev(f.ravel()), tol=1e-11)
    Uref = aa.bdf2_march(u0, f, aa.jacobian_A(alpha, 1.0, h, M), tau)
    print(f"tau1d M={M} Nt={Nt} bits={bits}: iters={st.iters}", flush=True)
    assert st.converged and st.true_rel_res <= 1e-11
    assert rel_max(to_host(U).reshape(Nt, M), Uref) < 1e-9


CASES_2D = [  # (alpha_x, alpha_y, Mx, My, Nt)
    (1.6, 1.4, 100, 60, 8),    # both axes chirp-z
    (1.5, 1.8, 60, 100, 5),
    (1.3, 1.7, 255, 60, 4),    # x on the FFT path, y chirp-z
    (1.7, 1.2, 100, 127, 6),   # x chirp-z, y on the FFT path
    (1.5, 1.5, 5, 3, 3),       # y on the FFT path (3 + 1 = 4), x chirp-z
    (1.9, 1.1, 1, 2, 2),
]


def _setup2d(gx, gy, Mx, My, Nt):
    hx, hy, tau = 1.0 / (Mx + 1), 1.0 / (My + 1), 1.0 / Nt
    Tx, Ty = aa.toeplitz_T(gx, Mx), aa.toeplitz_T(gy, My)
    cx, cy = twod.coeffs(gx, gy, 1.0, 1.0, hx, hy)
    return tau, Tx, Ty, cx, cy, pc.default_eps(tau)


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("gx,gy,Mx,My,Nt", CASES_2D)
def test_tau_preconditioner_any_length_2d(gx, gy, Mx, My, Nt, bits):
    from paper_2003_07020_amd.rfde import Plan
    banner(f"2d pinv any length bits={bits} {gx},{gy} {Mx}x{My} Nt={Nt}")
    p = Plan.create_2d(gx, gy, 1.0, 1.0, 0.0, 1.0, 0.0, 1.0, Mx, My, Nt, 1.0, precond_bits=bits)
    tau, Tx, Ty, cx, cy, eps = _setup2d(gx, gy, Mx, My, Nt)
    sx, sy = twod.tau_sigma_2d(gx, gy, Mx, My)
    v = wl.random_vector(53, Nt * My * Mx).reshape(Nt, My, Mx)
    z1 = pc.step_a(v.reshape(Nt, -1), eps).reshape(-1, My, Mx)
    z2 = to_host(p.step_b(to_dev(z1.ravel()))).reshape(z1.shape)
    ref = twod.step_b_tau_2d(z1, sx, sy, cx, cy, tau, Nt, eps)
    assert rel_max(z2, ref) < (1e-11 if bits == 64 else 2e-5)
    z = to_host(p.apply_Pinv(to_dev(v.ravel()))).reshape(v.shape)
    assert rel_max(z, twod.pinv_tau_2d(v, sx, sy, cx, cy, tau, eps)) < (1e-10 if bits == 64 else 1e-4)


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("gx,gy,Mx,My,Nt", CASES_2D[:4])
def test_solve_any_length_2d(gx, gy, Mx, My, Nt, bits):
    from paper_2003_07020_amd.rfde import Plan
    banner(f"2d solve any length bits={bits} {gx},{gy} {Mx}x{My} Nt={Nt}")
    p = Plan.create_2d(gx, gy, 1.0, 1.0, 0.0, 1.0, 0.0, 1.0, Mx, My, Nt, 1.0, precond_bits=bits)
    tau, Tx, Ty, cx, cy, eps = _setup2d(gx, gy, Mx, My, Nt)
    u0, f, _ = wl.gen2d(54, Mx, My, Nt)
    U, st, _ = p.solve(to_dev(u0.ravel()), to_dev(f.ravel()), tol=1e-11)
    assert st.converged and st.true_rel_res <= 1e-11
    Uref = twod.bdf2_march_2d(u0, f, Tx, Ty, cx, cy, tau)
    assert rel_max(to_host(U).reshape(Nt, My, Mx), Uref) < 1e-9
