"""Pins for the eps-circulant preconditioner (Section 3)."""
import numpy as np
import pytest
import scipy.fft as sfft
import scipy.linalg as sla

from oracle import allatonce as aa
from oracle import precond as pc
from oracle.weights import gk_recurrence


@pytest.mark.parametrize("Nt,eps", [(2, 0.25), (3, 0.5), (8, 0.5), (16, 1 / 32), (33, 0.01), (10, 1.0)])
def test_eigenvalues_match_dense_eig(Nt, eps):
    lam = pc.eigenvalues(Nt, eps)
    ev = np.linalg.eigvals(pc.C_eps_dense(Nt, eps))
    # match as multisets
    for l in lam:
        assert np.min(np.abs(ev - l)) < 1e-12
    for e in ev:
        assert np.min(np.abs(lam - e)) < 1e-12


@pytest.mark.parametrize("Nt,eps", [(8, 0.5), (16, 1 / 32), (7, 0.2)])
def test_diagonalization_identity(Nt, eps):
    # C_eps = V D V^{-1}, V = Lambda_eps F^*, Lambda_eps = diag(eps^{-j/N_t}) (eq. (3.2)-(3.3))
    F = pc.fourier_matrix(Nt)
    Lam = np.diag(1.0 / pc.scaling_s(Nt, eps))
    V = Lam @ F.conj().T
    D = np.diag(pc.eigenvalues(Nt, eps))
    assert np.allclose(V @ D @ np.linalg.inv(V), pc.C_eps_dense(Nt, eps), atol=1e-12)
    # D = diag(sqrt(N_t) F Lambda^{-1} C_eps(:, 1))
    d = np.sqrt(Nt) * F @ np.linalg.inv(Lam) @ pc.C_eps_dense(Nt, eps)[:, 0]
    assert np.allclose(d, pc.eigenvalues(Nt, eps), atol=1e-12)


@pytest.mark.parametrize("Nt", (8, 64, 1024))
def test_proposition_3_1(Nt):
    # Re lambda_n >= 0, with equality only for eps = 1 (then lambda_0 = 0)
    for eps in (0.5, 1 / (2 * Nt), 1e-3):
        lam = pc.eigenvalues(Nt, eps)
        assert np.all(lam.real > 0)
        # closed form of the real part: (1/2)[(1 - x)(3 - x) - y^2], x + iy = eps^{1/N_t} theta^n
        z = eps ** (1 / Nt) * np.exp(2j * np.pi * np.arange(Nt) / Nt)
        x, y = z.real, z.imag
        assert np.allclose(lam.real, 0.5 * ((1 - x) * (3 - x) - y**2), atol=1e-13)
    lam1 = pc.eigenvalues(Nt, 1.0)
    assert abs(lam1[0]) < 1e-14
    assert np.all(lam1.real > -1e-14)


def test_step_a_is_the_fourier_matrix_product():
    Nt, M, eps = 12, 5, 0.3
    v = np.random.default_rng(1).standard_normal((Nt, M))
    F = pc.fourier_matrix(Nt)
    z1 = np.sqrt(Nt) * F @ (pc.scaling_s(Nt, eps)[:, None] * v)
    assert np.allclose(pc.step_a(v, eps), z1[: Nt // 2 + 1], atol=1e-12)


@pytest.mark.parametrize("gam,Nt,M,eps", [(1.5, 8, 7, None), (1.2, 10, 6, 0.2),
                                          (1.8, 16, 5, None), (1.5, 9, 4, 1.0),
                                          (1.5, 2, 6, None), (1.3, 3, 5, None)])
def test_fast_pinv_equals_dense_inverse(gam, Nt, M, eps):
    h, tau = aa.mesh(0, 1, M, 1.0, Nt)
    eps = pc.default_eps(tau) if eps is None else eps
    A = aa.jacobian_A(gam, 1.0, h, M)
    v = np.random.default_rng(2).standard_normal((Nt, M))
    zd = pc.pinv_dense(v, A, tau, eps)
    zf = pc.pinv_fast(v, A, tau, eps)
    assert np.max(np.abs(zf - zd)) < 1e-12 * np.max(np.abs(zd))
    # the imaginary part of step (c) vanishes (conjugate-symmetric spectrum)
    z2 = pc.step_b_exact(pc.step_a(v, eps), A, tau, Nt, eps)
    zc = pc.step_c_complex(z2, Nt, eps)
    assert np.max(np.abs(zc.imag)) < 1e-12 * np.max(np.abs(zc.real))


def test_conjugate_symmetry_of_shifted_solutions():
    # z2_{N_t-n} = conj(z2_n) (Section 3.2): solve ALL N_t systems and compare
    gam, Nt, M = 1.5, 10, 6
    h, tau = aa.mesh(0, 1, M, 1.0, Nt)
    eps = pc.default_eps(tau)
    A = aa.jacobian_A(gam, 1.0, h, M)
    v = np.random.default_rng(3).standard_normal((Nt, M))
    w = pc.scaling_s(Nt, eps)[:, None] * v
    z1 = Nt * sfft.ifft(w, axis=0)
    lam = pc.eigenvalues(Nt, eps)
    z2 = np.array([np.linalg.solve(pc.shifted_matrix(lam[n], A, tau), z1[n]) for n in range(Nt)])
    for n in range(1, Nt):
        assert np.allclose(z2[Nt - n], np.conj(z2[n]), atol=1e-13)
    assert pc.n_unique(Nt) == Nt // 2 + 1 == 6


@pytest.mark.parametrize("gam,Nt,M", [(1.5, 8, 6), (1.2, 12, 5), (1.8, 16, 4)])
def test_rank_and_clustering(gam, Nt, M):
    # Theorem 3.1 (corrected): P^{-1} A - I = P^{-1} ((C - C_eps) kron I_s) has rank 2 N_s
    # (the printed 2 N_t counts time blocks, but C - C_eps has 2 nonzero columns of
    # blocks each of rank N_s); so >= (N_t - 2) N_s eigenvalues equal 1.
    h, tau = aa.mesh(0, 1, M, 1.0, Nt)
    eps = pc.default_eps(tau)
    A = aa.jacobian_A(gam, 1.0, h, M)
    Aall = aa.all_at_once_matrix(aa.time_matrix_C(Nt), A, tau)
    P = pc.preconditioner_dense(A, tau, Nt, eps)
    L = np.linalg.solve(P, Aall) - np.eye(Nt * M)
    s = np.linalg.svd(L, compute_uv=False)
    rank = int(np.sum(s > 1e-10 * s[0]))
    assert rank == 2 * M
    ev = np.linalg.eigvals(np.linalg.solve(P, Aall))
    assert np.sum(np.abs(ev - 1) < 1e-8) >= (Nt - 2) * M


def test_dst_matrix_and_library_dst():
    for n in (1, 5, 16):
        Q = pc.dst_matrix(n)
        assert np.allclose(Q, Q.T)
        assert np.allclose(Q @ Q, np.eye(n), atol=1e-14)
        x = np.random.default_rng(n).standard_normal(n)
        assert np.allclose(sfft.dst(x, type=1, norm="ortho"), Q @ x, atol=1e-14)


@pytest.mark.parametrize("gam", (1.2, 1.5, 1.9))
def test_tau_matrix_is_toeplitz_minus_hankel(gam):
    # The natural tau approximation of a symmetric Toeplitz T (Bini-Di Benedetto) is T - H
    # with the persymmetric Hankel H whose first row is (t_2, ..., t_{n-1}, 0, 0) and last
    # row its reverse: H[i, j] = t_{i+j+2} if i+j+2 <= n-1, t_{2n-i-j} if i+j >= n+1, else 0
    # (0-based).  This is an independent definition of the same matrix.
    n = 9
    t = gk_recurrence(gam, n)

    def hank(i, j):
        if i + j + 2 <= n - 1:
            return t[i + j + 2]
        if i + j >= n + 1:
            return t[2 * n - i - j]
        return 0.0

    H = np.array([[hank(i, j) for j in range(n)] for i in range(n)])
    assert np.allclose(pc.tau_matrix(t), sla.toeplitz(t) - H, atol=1e-14)


def test_tau_eigenvalues_gamma_two():
    # gamma = 2: T is tridiagonal (2, -1), already a tau matrix; sigma_i = 2 - 2 cos(pi i/(n+1))
    n = 17
    sig = pc.tau_eigenvalues(gk_recurrence(2.0, n))
    i = np.arange(1, n + 1)
    assert np.allclose(sig, 2 - 2 * np.cos(np.pi * i / (n + 1)), atol=1e-13)


def test_printed_pattern_for_three_or_more_steps():
    # for N_t >= 3, r(Z_eps) is the matrix drawn in eq. (3.1)
    Nt, eps = 6, 0.3
    Ce = pc.C_eps_dense(Nt, eps)
    c = np.array([1.5, -2.0, 0.5, 0, 0, 0])
    for j in range(Nt):
        for k in range(Nt):
            assert Ce[j, k] == (c[j - k] if j >= k else eps * c[j - k + Nt])


def test_default_eps():
    assert pc.default_eps(1 / 64) == 1 / 128
    assert pc.default_eps(2.0) == 0.5
