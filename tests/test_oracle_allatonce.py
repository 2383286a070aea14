"""Pins for the Toeplitz block, the BDF2 all-at-once system and its properties (Section 2)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import allatonce as aa
from oracle.weights import gk_recurrence
from rfde_workloads import gen1d


@pytest.mark.parametrize("gam", (1.2, 1.5, 1.8))
def test_toeplitz_spd_and_spectrum(gam):
    # T_x is SPD (Section 2.1); its eigenvalues lie strictly inside the range of the
    # symbol |2 sin(theta/2)|^gam, i.e. in (0, 2^gam)
    T = aa.toeplitz_T(gam, 120)
    assert np.allclose(T, T.T)
    sla.cholesky(T)  # raises if not positive definite
    ev = np.linalg.eigvalsh(T)
    assert ev.min() > 0 and ev.max() < 2**gam


def test_time_matrix_and_inverse_closed_form():
    # Lemma 2.3 proof: explicit C^{-1}; first column 1, 4/3, 13/9, 40/27, ...
    for Nt in (2, 3, 7, 33):
        C = aa.time_matrix_C(Nt)
        assert np.allclose(np.linalg.inv(C), aa.C_inverse_closed_form(Nt), atol=1e-13)
    Ci = aa.C_inverse_closed_form(6)
    assert np.allclose(Ci[:4, 0], [1, 4 / 3, 13 / 9, 40 / 27])


@pytest.mark.parametrize("Nt", (4, 16, 64))
def test_lemma_2_3_norm_values(Nt):
    # Lemma 2.3 values; the printed norm labels are swapped: the maximum ROW sum of C^{-1}
    # is N_t and the maximum COLUMN sum is 3 N_t / 2 - 3/4 (1 - 3^{-N_t})
    Ci = np.linalg.inv(aa.time_matrix_C(Nt))
    assert np.isclose(np.abs(Ci).sum(axis=1).max(), Nt, rtol=1e-12)
    assert np.isclose(np.abs(Ci).sum(axis=0).max(), 1.5 * Nt - 0.75 * (1 - 3.0**-Nt), rtol=1e-12)
    C = aa.time_matrix_C(Nt)
    # ||C||_1 = ||C||_inf = 4 (Theorem 2.1 proof) once N_t >= 3
    assert np.isclose(np.abs(C).sum(axis=0).max(), 4.0)
    assert np.isclose(np.abs(C).sum(axis=1).max(), 4.0)


@pytest.mark.parametrize("gam,Nt,M", [(1.5, 8, 6), (1.2, 12, 5), (1.8, 6, 9)])
def test_theorem_2_1_bounds(gam, Nt, M):
    # advisory: the singular-value bounds of Theorem 2.1 on small cases
    h, tau = aa.mesh(0, 1, M, 1.0, Nt)
    A = aa.jacobian_A(gam, 1.0, h, M)
    Aall = aa.all_at_once_matrix(aa.time_matrix_C(Nt), A, tau)
    s = np.linalg.svd(Aall, compute_uv=False)
    assert s.max() <= 4 + tau * np.linalg.norm(A, 2) + 1e-12
    assert s.min() >= np.sqrt(6) / (3 * Nt) - 1e-12


def test_matvec_equals_dense_kron():
    gam, Nt, M = 1.5, 9, 7
    h, tau = aa.mesh(0, 1, M, 1.0, Nt)
    A = aa.jacobian_A(gam, 1.0, h, M)
    v = np.random.default_rng(0).standard_normal((Nt, M))
    dense = aa.all_at_once_matrix(aa.time_matrix_C(Nt), A, tau) @ v.ravel()
    assert np.allclose(aa.apply_all_at_once(v, A, tau).ravel(), dense, rtol=1e-14, atol=1e-13)
    # the Kronecker product ordering itself: block (k, j) = C[k, j] I - tau delta_kj A
    Aall = aa.all_at_once_matrix(aa.time_matrix_C(Nt), A, tau)
    assert np.allclose(Aall[M:2 * M, 0:M], -2.0 * np.eye(M))
    assert np.allclose(Aall[2 * M:3 * M, 2 * M:3 * M], 1.5 * np.eye(M) - tau * A)


@pytest.mark.parametrize("gam", (1.2, 1.5, 1.8))
def test_march_equals_dense_solve(gam):
    # C lower triangular => the all-at-once solution is the sequential BDF2 march
    Nt, M = 16, 15
    h, tau = aa.mesh(0, 1, M, 1.0, Nt)
    A = aa.jacobian_A(gam, 1.0, h, M)
    u0, f, _ = gen1d(7, M, Nt)
    U1 = aa.bdf2_march(u0, f, A, tau)
    U2 = aa.dense_direct(u0, f, A, tau)
    U3 = aa.bdf2_march_eig(u0, f, A, tau)
    assert np.max(np.abs(U1 - U2)) < 1e-13 * np.max(np.abs(U2))
    assert np.max(np.abs(U3 - U2)) < 1e-12 * np.max(np.abs(U2))
    # residual of the assembled system
    Aall = aa.all_at_once_matrix(aa.time_matrix_C(Nt), A, tau)
    F = aa.rhs_F(u0, f, tau).ravel()
    assert np.linalg.norm(Aall @ U1.ravel() - F) < 1e-13 * np.linalg.norm(F)


def test_rhs_first_two_levels():
    # eq. (2.11): F_1 = tau f^1 + u^0, F_2 = tau f^2 - u^0 / 2, F_k = tau f^k
    u0 = np.arange(3.0)
    f = np.ones((4, 3))
    F = aa.rhs_F(u0, f, 0.25)
    assert np.allclose(F[0], 0.25 + u0)
    assert np.allclose(F[1], 0.25 - 0.5 * u0)
    assert np.allclose(F[2:], 0.25)
