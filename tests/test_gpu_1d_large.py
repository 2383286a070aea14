"""GPU parity at the full benchmarked 1D shape (M = 4095, N_t = 1024, 513 shifted blocks), in the
launch configuration bench.py times: every output of the cheap steps element by element, the
shifted solves on sampled frequencies, the preconditioner through the identity P z = v, and the
solve against the oracle's sequential BDF2 march."""
import numpy as np
import pytest
import scipy.linalg as sla

from gpu_util import TOL_FFT, banner, rel_max, to_dev, to_host
from oracle import allatonce as aa
from oracle import precond as pc
from oracle.weights import gk_recurrence
from rfde_workloads import LARGE_1D, gen1d, random_vector

pytestmark = pytest.mark.gpu

M, NT, KAPPA, T = LARGE_1D["M"], LARGE_1D["Nt"], LARGE_1D["kappa"], LARGE_1D["T"]


@pytest.fixture(scope="module", params=[1.8])
def big(request):
    from paper_2003_07020_amd.rfde import Plan
    alpha = request.param
    banner(f"large plan alpha={alpha} M={M} Nt={NT}")
    p = Plan.create_1d(alpha, KAPPA, 0.0, 1.0, M, NT, T, tol=1e-10)
    h, tau = aa.mesh(0.0, 1.0, M, T, NT)
    A = aa.jacobian_A(alpha, KAPPA, h, M)
    yield alpha, p, h, tau, A, pc.default_eps(tau)
    p.destroy()


def test_setup_arrays(big):
    from paper_2003_07020_amd import capi
    alpha, p, h, tau, A, eps = big
    g = to_host(p.export(capi.EXPORT_GK))
    assert rel_max(g, gk_recurrence(alpha, M)) < 1e-12
    L = p.info["L"]
    assert L == 8192
    sym = to_host(p.export(capi.EXPORT_SYMBOL))
    ref = aa.circulant_symbol(gk_recurrence(alpha, M), M, L)[: L // 2 + 1] * p.info["coef"] / L
    assert rel_max(sym, ref) < TOL_FFT
    lam = to_host(p.export(capi.EXPORT_LAMBDA))
    assert rel_max(lam, pc.eigenvalues(NT, eps)[: NT // 2 + 1]) < 1e-14


def test_matvec_full(big):
    alpha, p, h, tau, A, eps = big
    v = random_vector(21, NT * M).reshape(NT, M)
    y = to_host(p.apply_A(to_dev(v.ravel()))).reshape(NT, M)
    assert rel_max(y, aa.apply_all_at_once(v, A, tau)) < TOL_FFT


def test_time_steps_full(big):
    alpha, p, h, tau, A, eps = big
    v = random_vector(22, NT * M).reshape(NT, M)
    z1 = to_host(p.step_a(to_dev(v.ravel()))).reshape(-1, M)
    z1_ref = pc.step_a(v, eps)
    assert rel_max(z1, z1_ref) < TOL_FFT
    zc = to_host(p.step_c(to_dev(z1_ref.ravel()))).reshape(NT, M)
    assert rel_max(zc, pc.step_c(z1_ref, NT, eps)) < TOL_FFT


def test_shifted_solves_sampled(big):
    alpha, p, h, tau, A, eps = big
    v = random_vector(23, NT * M).reshape(NT, M)
    z1_ref = pc.step_a(v, eps)
    z2 = to_host(p.step_b(to_dev(z1_ref.ravel()))).reshape(-1, M)
    lam = pc.eigenvalues(NT, eps)
    for n in (0, 1, 300, NT // 2):
        B = pc.shifted_matrix(lam[n], A, tau)
        ref = sla.lu_solve(sla.lu_factor(B), z1_ref[n])
        # forward error: cond(B_0) ~ 7e5 at alpha = 1.8 (smallest eigenvalue Re lambda_0 +
        # coef lambda_min(T) ~ 0.015, largest ~ 1.1e4), so each solver is accurate to about
        # cond * u * sqrt(M) ~ 5e-9; allow 2e-8 between them
        assert rel_max(z2[n], ref) < 2e-8, n
        # normwise backward error of the GPU solution itself (the decisive check); the
        # Wilkinson-type bound for an order-M elimination and residual is ~ M u = 4.5e-13
        bwd = np.linalg.norm(B @ z2[n] - z1_ref[n]) / (
            np.linalg.norm(B, 1) * np.linalg.norm(z2[n]) + np.linalg.norm(z1_ref[n]))
        assert bwd < 1e-13, (n, bwd)


def test_preconditioner_identity(big):
    # P_eps z = v with P_eps = C_eps kron I + I kron (coef T): check every entry of the residual
    alpha, p, h, tau, A, eps = big
    v = random_vector(24, NT * M).reshape(NT, M)
    z = to_host(p.apply_Pinv(to_dev(v.ravel()))).reshape(NT, M)
    Pz = np.empty_like(z)
    for k in range(NT):
        Pz[k] = 1.5 * z[k] - 2.0 * (z[k - 1] if k >= 1 else eps * z[NT - 1]) \
            + 0.5 * (z[k - 2] if k >= 2 else eps * z[NT - 2 + k])
    Pz -= tau * (z @ A.T)
    # a backward-stable apply leaves ||P z - v|| <~ c u ||P|| ||z||, with ||P|| ~ 1.1e4 and
    # ||z|| <~ ||v|| / 0.015 here: ~7e-11 c, so allow 1e-8
    assert rel_max(Pz, v) < 1e-8


@pytest.fixture(scope="module")
def march(big):
    # the oracle's sequential BDF2 march of one seeded problem (about 10 s on the host)
    alpha, p, h, tau, A, eps = big
    u0, f, _ = gen1d(2000 + 2, M, NT)
    return u0, f, aa.bdf2_march(u0, f, A, tau)


def test_solve_full(big, march):
    alpha, p, h, tau, A, eps = big
    u0, f, Uref = march
    U, st, _ = p.solve(to_dev(u0), to_dev(f.ravel()), tol=1e-10)
    U = to_host(U).reshape(NT, M)
    assert st.converged and st.true_rel_res <= 1e-10
    assert rel_max(U, Uref) < 1e-8


def test_solve_full_tau(big, march):
    # the paper's step (b) (tau/DST-I, the half-length transform at this size) at the
    # benchmarked shape: the preconditioner differs, the solution of the all-at-once system
    # does not
    from paper_2003_07020_amd.rfde import Plan
    alpha, _, h, tau, A, eps = big
    u0, f, Uref = march
    banner(f"large tau solve alpha={alpha}")
    with Plan.create_1d(alpha, KAPPA, 0.0, 1.0, M, NT, T, tol=1e-10, spatial="tau") as q:
        U, st, _ = q.solve(to_dev(u0), to_dev(f.ravel()))
    print(f"tau at M={M}, Nt={NT}: iters={st.iters} true_rel_res={st.true_rel_res:.2e}",
          flush=True)
    assert st.converged and st.true_rel_res <= 1e-10
    assert rel_max(to_host(U).reshape(NT, M), Uref) < 1e-8
