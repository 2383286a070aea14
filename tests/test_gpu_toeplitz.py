"""GPU parity of the factor-free exact step (b) (spatial = "toeplitz"): the Levinson-Durbin
generators (first columns of the shifted-block inverses) and the Gohberg-Semencul solves against
the oracle's dense solves, P^-1 against the oracle's fast P^-1, and full solves against the
oracle's march; the preconditioner is the exact one, so the iteration counts match the LDL^T
form's."""
import numpy as np
import pytest
import scipy.linalg as sla

from gpu_util import banner, rel_max, to_dev, to_host
from oracle import allatonce as aa
from oracle import precond as pc
import rfde_workloads as wl

pytestmark = pytest.mark.gpu


def _plan(alpha, M, Nt, **kw):
    from paper_2003_07020_amd.rfde import Plan
    return Plan.create_1d(alpha, 1.0, 0.0, 1.0, M, Nt, 1.0, spatial="toeplitz", **kw)


@pytest.mark.parametrize("alpha,M,Nt", [(1.5, 1, 2), (1.3, 2, 4), (1.7, 7, 3), (1.5, 63, 16),
                                        (1.8, 100, 7), (1.2, 1000, 8), (1.9, 255, 64),
                                        (1.4, 300, 6), (1.6, 2000, 4), (1.3, 4096, 4),
                                        # orders whose pair count crosses a thread-slot
                                        # boundary of the setup (256 pairs per slot)
                                        (1.5, 515, 6), (1.7, 1026, 5), (1.2, 1539, 4)])
def test_generators_and_shifted_solves(alpha, M, Nt):
    from paper_2003_07020_amd import capi
    banner(f"toeplitz small alpha={alpha} M={M} Nt={Nt}")
    p = _plan(alpha, M, Nt)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    A = aa.jacobian_A(alpha, 1.0, h, M)
    eps = pc.default_eps(tau)
    lam = pc.eigenvalues(Nt, eps)
    for n in sorted({0, 1, Nt // 4, Nt // 2}):
        B = pc.shifted_matrix(lam[n], A, tau)
        x = to_host(p.export(capi.EXPORT_TOEPLITZ_X, n))
        xr = sla.lu_solve(sla.lu_factor(B), np.eye(M)[:, 0])
        # the generator is B^-1 e_0: its accuracy is cond(B) u at most
        assert rel_max(x, xr) < max(1e-12, 1e-15 * np.linalg.cond(B)), n
    v = wl.random_vector(61, Nt * M).reshape(Nt, M)
    z1 = pc.step_a(v, eps)
    z2 = to_host(p.step_b(to_dev(z1.ravel()))).reshape(-1, M)
    assert rel_max(z2, pc.step_b_exact(z1, A, tau, Nt, eps)) < 1e-10
    z = to_host(p.apply_Pinv(to_dev(v.ravel()))).reshape(Nt, M)
    assert rel_max(z, pc.pinv_fast(v, A, tau, eps)) < 1e-10


@pytest.mark.parametrize("alpha,M,Nt", [(1.5, 2100, 512), (1.7, 2049, 513), (1.6, 4096, 512)])
def test_shifted_solves_last_row_direct(alpha, M, Nt):
    """257 frequency rows at transform length 8192 (one workgroup per CU): on a 256-CU device the
    last row is formed by direct sums spread over the other rows' workgroups instead of a round
    of its own (at M = 4096 its two staged vectors fill the transform buffer exactly).  Sampled
    rows, the last included, against dense solves."""
    banner(f"toeplitz last row alpha={alpha} M={M} Nt={Nt}")
    p = _plan(alpha, M, Nt)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    A = aa.jacobian_A(alpha, 1.0, h, M)
    eps = pc.default_eps(tau)
    lam = pc.eigenvalues(Nt, eps)
    nf = Nt // 2 + 1
    v = wl.random_vector(63, Nt * M).reshape(Nt, M)
    z1 = pc.step_a(v, eps)
    z2 = to_host(p.step_b(to_dev(z1.ravel()))).reshape(-1, M)
    for n in (0, 1, nf // 2, nf - 2, nf - 1):
        ref = sla.lu_solve(sla.lu_factor(pc.shifted_matrix(lam[n], A, tau)), z1[n])
        assert rel_max(z2[n], ref) < 1e-10, n


@pytest.mark.parametrize("alpha,M,Nt", [(1.5, 63, 64), (1.8, 1023, 16), (1.3, 100, 9)])
def test_solve_matches_march_and_exact_iterations(alpha, M, Nt):
    from paper_2003_07020_amd.rfde import Plan
    banner(f"toeplitz solve alpha={alpha} M={M} Nt={Nt}")
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    u0, f, _ = wl.gen1d(62, M, Nt)
    Uref = aa.bdf2_march(u0, f, aa.jacobian_A(alpha, 1.0, h, M), tau)
    with _plan(alpha, M, Nt, tol=1e-11) as p:
        U, st, _ = p.solve(to_dev(u0), to_dev(f.ravel()))
    assert st.converged and st.true_rel_res <= 1e-11
    assert rel_max(to_host(U).reshape(Nt, M), Uref) < 1e-9
    with Plan.create_1d(alpha, 1.0, 0.0, 1.0, M, Nt, 1.0, tol=1e-11) as q:
        _, st2, _ = q.solve(to_dev(u0), to_dev(f.ravel()))
    # the same exact preconditioner: the counts may differ only by rounding
    assert abs(st.iters - st2.iters) <= 1, (st.iters, st2.iters)


def test_fp32_toeplitz_is_unsupported():
    from paper_2003_07020_amd import capi
    with pytest.raises(capi.RfdeError) as e:
        _plan(1.5, 63, 16, precond_bits=32)
    assert e.value.code == capi.RFDE_EUNSUPPORTED
