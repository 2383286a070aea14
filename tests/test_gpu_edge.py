"""GPU edge cases: degenerate parameters of the method, limits of the ABI, error paths that a
caller can trigger from the host, and bitwise reproducibility."""
import numpy as np
import pytest

from gpu_util import banner, rel_max, to_dev, to_host
from oracle import allatonce as aa
from oracle import precond as pc
from rfde_workloads import gen1d, random_vector

pytestmark = pytest.mark.gpu


def _plan(alpha, kappa, M, Nt, **kw):
    from paper_2003_07020_amd.rfde import Plan
    return Plan.create_1d(alpha, kappa, 0.0, 1.0, M, Nt, 1.0, **kw)


def _check_solve(alpha, kappa, M, Nt, tol=1e-10, **kw):
    p = _plan(alpha, kappa, M, Nt, tol=tol, **kw)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    u0, f, _ = gen1d(21, M, Nt)
    U, st, _ = p.solve(to_dev(u0), to_dev(f.ravel()))
    Uref = aa.bdf2_march(u0, f, aa.jacobian_A(alpha, kappa, h, M), tau)
    assert st.converged and st.true_rel_res <= tol
    assert rel_max(to_host(U).reshape(Nt, M), Uref) < 1e-8
    return st


def test_gamma_two_classical_diffusion():
    # Lemma 2.2: alpha = 2 is the three-point Laplacian; the path must handle g = (2, -1, 0, ...)
    banner("alpha=2")
    _check_solve(2.0, 1.0, 100, 16)


def test_bc_preconditioner_eps_one():
    # eps = 1: the BC preconditioner P_1 (Remark 3.1), lambda_0 = 0 (Proposition 3.1)
    banner("eps=1")
    st1 = _check_solve(1.5, 1.0, 63, 32, circ_eps=1.0)
    st = _check_solve(1.5, 1.0, 63, 32)
    assert st1.iters >= st.iters


def test_long_arnoldi_cycle():
    # more than 16 Arnoldi steps in one restart cycle: the Gram-Schmidt sweeps then split the
    # basis into chunks of 16 dot products (tau step (b), which is inexact, at tight tolerances)
    banner("long Arnoldi cycle")
    iters = []
    for alpha, M, Nt, tol, bits in ((1.05, 1023, 16, 1e-13, 64), (1.1, 511, 64, 1e-12, 32)):
        p = _plan(alpha, 1.0, M, Nt, tol=tol, spatial="tau", precond_bits=bits, restart=40)
        h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
        u0, f, _ = gen1d(21, M, Nt)
        U, st, _ = p.solve(to_dev(u0), to_dev(f.ravel()))
        Uref = aa.bdf2_march(u0, f, aa.jacobian_A(alpha, 1.0, h, M), tau)
        assert st.converged and st.true_rel_res <= tol
        assert rel_max(to_host(U).reshape(Nt, M), Uref) < 1e-9
        iters.append(st.iters)
    assert max(iters) > 16, iters


def test_tiny_kappa_and_single_point():
    banner("kappa tiny, M=1")
    _check_solve(1.5, 1e-6, 31, 8)
    _check_solve(1.7, 1.0, 1, 4)


def test_max_M_and_long_time_axis():
    banner("M=4096 Nt=2; M=15 Nt=8192")
    _check_solve(1.5, 1.0, 4096, 2)
    p = _plan(1.3, 1.0, 15, 8192)
    h, tau = aa.mesh(0.0, 1.0, 15, 1.0, 8192)
    v = random_vector(5, 8192 * 15).reshape(8192, 15)
    eps = pc.default_eps(tau)
    z1 = to_host(p.step_a(to_dev(v.ravel()))).reshape(-1, 15)
    assert rel_max(z1, pc.step_a(v, eps)) < 1e-12
    _check_solve(1.3, 1.0, 15, 8192)


def test_plan_too_large_is_enomem():
    from paper_2003_07020_amd import _lib as capi
    from paper_2003_07020_amd.rfde import Plan
    banner("ENOMEM")
    # 4097 blocks of 2080 tiles x 64 KiB = 558 GB of FP64 factors: rejected before allocation
    with pytest.raises(capi.RfdeError) as ei:
        Plan.create_1d(1.5, 1.0, 0.0, 1.0, 4096, 8192, 1.0)
    assert ei.value.code == capi.RFDE_ENOMEM


def test_zero_rhs_nan_rhs_and_maxit():
    from paper_2003_07020_amd import _lib as capi
    banner("zero/NaN rhs, maxit")
    M, Nt = 63, 16
    p = _plan(1.5, 1.0, M, Nt, tol=1e-12, maxit=2)
    u0, f, _ = gen1d(3, M, Nt)
    U, st, rc = p.solve(to_dev(np.zeros(M)), to_dev(np.zeros(Nt * M)))
    assert rc == capi.RFDE_OK and st.iters == 0 and np.all(to_host(U) == 0)
    bad = f.ravel().copy()
    bad[17] = np.nan
    with pytest.raises(capi.RfdeError) as ei:
        p.solve(to_dev(u0), to_dev(bad))
    assert ei.value.code == capi.RFDE_ENAN
    U, st, rc = p.solve(to_dev(u0), to_dev(f.ravel()), allow_notconv=True)
    assert rc == capi.RFDE_ENOTCONV and st.iters == 2 and not st.converged


def test_exact_initial_guess_needs_no_iteration():
    banner("exact guess")
    M, Nt, alpha = 63, 16, 1.5
    p = _plan(alpha, 1.0, M, Nt, tol=1e-10)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    u0, f, _ = gen1d(4, M, Nt)
    Uref = aa.bdf2_march(u0, f, aa.jacobian_A(alpha, 1.0, h, M), tau)
    U, st, _ = p.solve(to_dev(u0), to_dev(f.ravel()), U_init=to_dev(Uref.ravel()))
    assert st.converged and st.iters == 0


@pytest.mark.parametrize("restart", [1, 17, 64])
def test_arnoldi_cycle_lengths(restart):
    # FGMRES(1) (a factor of order 1 in every cycle), FGMRES(17) (its last step projects onto
    # 17 stored vectors, one past the 16 dot products of a sweep) and FGMRES(64): the
    # solution matches the oracle's BDF2 march, and the residual estimate of the last step
    # agrees with the true residual, which holds only if A Z = V H with the implicit
    # orthonormal basis
    banner(f"arnoldi cycle restart={restart}")
    if restart == 1:
        alpha, M, Nt, tol, kw = 1.5, 63, 16, 1e-10, dict(maxit=400)
    else:
        alpha, M, Nt, tol, kw = 1.05, 1023, 16, 1e-13, dict(spatial="tau")
    p = _plan(alpha, 1.0, M, Nt, tol=tol, restart=restart, **kw)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    u0, f, _ = gen1d(21, M, Nt)
    U, st, _ = p.solve(to_dev(u0), to_dev(f.ravel()))
    Uref = aa.bdf2_march(u0, f, aa.jacobian_A(alpha, 1.0, h, M), tau)
    print(f"restart={restart}: iters={st.iters} restarts={st.restarts} "
          f"est={st.res_hist[-1]:.3e} true={st.true_rel_res:.3e}", flush=True)
    assert st.converged and st.true_rel_res <= tol
    assert rel_max(to_host(U).reshape(Nt, M), Uref) < 1e-9
    assert abs(np.log10(st.res_hist[-1]) - np.log10(st.true_rel_res)) < 0.5
    if restart == 1:
        assert st.restarts == st.iters
    else:
        assert st.iters >= 17


def test_restart_path_converges():
    banner("restart m=2")
    st = _check_solve(1.8, 1.0, 100, 32, restart=2, maxit=200)
    assert st.restarts >= 2


def test_bitwise_reproducible():
    banner("reproducibility")
    M, Nt = 200, 32
    p = _plan(1.5, 1.0, M, Nt)
    u0, f, _ = gen1d(9, M, Nt)
    U1, st1, _ = p.solve(to_dev(u0), to_dev(f.ravel()))
    U2, st2, _ = p.solve(to_dev(u0), to_dev(f.ravel()))
    q = _plan(1.5, 1.0, M, Nt)
    U3, st3, _ = q.solve(to_dev(u0), to_dev(f.ravel()))
    a, b, c = to_host(U1), to_host(U2), to_host(U3)
    assert np.array_equal(a, b) and np.array_equal(a, c)
    assert st1.res_hist == st2.res_hist == st3.res_hist


def test_one_call_solve():
    from paper_2003_07020_amd import rfde
    banner("rfde.solve")
    M, Nt, alpha, kappa = 50, 12, 1.4, 0.9
    u0, f, _ = gen1d(31, M, Nt)
    U, st = rfde.solve(alpha, kappa, (0.0, 1.0), M, Nt, 1.0, to_dev(u0), to_dev(f.ravel()),
                       tol=1e-11)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    assert st.converged
    assert rel_max(to_host(U).reshape(Nt, M),
                   aa.bdf2_march(u0, f, aa.jacobian_A(alpha, kappa, h, M), tau)) < 1e-9


def test_device_memory_cache_reuse_and_release():
    from paper_2003_07020_amd import rfde
    banner("memory cache")
    rfde.release_cached_memory()
    p = _plan(1.5, 1.0, 300, 64)
    ptr_bytes = p.info["factor_bytes"]
    p.destroy()
    # the freed blocks are cached, a second plan of the same shape reuses them and is correct
    _check_solve(1.5, 1.0, 300, 64)
    released = rfde.release_cached_memory()
    assert released >= ptr_bytes
    assert rfde.release_cached_memory() == 0
