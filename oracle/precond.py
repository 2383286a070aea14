"""The alpha-circulant (here: eps-circulant) preconditioner P_eps = C_eps kron I - tau I kron A.

Section 3.1 (eq. (3.1)-(3.4)) and Section 3.2.  The paper calls the circulant
parameter alpha; the library reserves `alpha` for the fractional order, so it is
`eps` here.  The default is eps = min(0.5, 0.5 tau) (Section 4).

Sign convention: the Fourier matrix of eq. (3.3) uses theta = exp(+2 pi i / N_t).
Step (a) therefore computes z1_n = sum_j theta^{n j} s_j v_j (numpy: N_t * ifft over
time) and step (c) v_j = s_j^{-1} (1/N_t) sum_n theta^{-n j} z2_n (numpy: fft / N_t);
the 1/sqrt(N_t) factors of the unitary matrix cancel between the two steps.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla

R_COEF = (1.5, -2.0, 0.5)  # r_0, r_1, r_2 of eq. (3.3): first column of C_eps


def default_eps(tau: float) -> float:
    """eps = min(0.5, 0.5 tau) (Section 4, first paragraph)."""
    return min(0.5, 0.5 * tau)


def C_eps_dense(Nt: int, eps: float) -> np.ndarray:
    """C_eps of eq. (3.1): the Strang-type eps-circulant built from C's Toeplitz part,
    r(Z) = 3/2 I - 2 Z + 1/2 Z^2 with Z the eps-circulant down-shift (Z e_j = e_{j+1},
    Z e_{N_t-1} = eps e_0).  For N_t >= 3 this is exactly the printed matrix:
    C_eps[j, k] = c_{j-k} (j >= k), eps c_{j-k+N_t} (j < k), c = (3/2, -2, 1/2, 0, ...).
    Reading for N_t = 2 (the printed pattern needs N_t >= 3): Z^2 = eps I, so the 1/2 term
    wraps onto the diagonal; this is the matrix whose eigenvalues eq. (3.3) gives."""
    Z = np.zeros((Nt, Nt))
    for j in range(Nt - 1):
        Z[j + 1, j] = 1.0
    Z[0, Nt - 1] = eps
    out = np.zeros((Nt, Nt))
    P = np.eye(Nt)
    for r in R_COEF:
        out += r * P
        P = Z @ P
    return out


def scaling_s(Nt: int, eps: float) -> np.ndarray:
    """s_j = eps^{j/N_t}, j = 0..N_t-1: the diagonal of Lambda_eps^{-1} in eq. (3.3).
    Each power is exp((j/N_t) ln eps) evaluated independently (no running product)."""
    j = np.arange(Nt, dtype=np.float64)
    return np.exp((j / Nt) * np.log(eps))


def eigenvalues(Nt: int, eps: float) -> np.ndarray:
    """lambda_n = sum_{j=0}^{2} r_j eps^{j/N_t} theta^{n j}, n = 0..N_t-1 (eq. (3.3))."""
    n = np.arange(Nt)
    lam = np.zeros(Nt, dtype=np.complex128)
    for j, r in enumerate(R_COEF):
        # theta^{n j} = exp(2 pi i ((n j) mod N_t) / N_t): the exact integer reduction keeps the
        # angle correctly rounded (repeated powers of theta lose about n j ulps)
        lam += r * eps ** (j / Nt) * np.exp(2j * np.pi * ((n * j) % Nt) / Nt)
    return lam


def fourier_matrix(Nt: int) -> np.ndarray:
    """Unitary F_{N_t} of eq. (3.3): F[j, k] = theta^{j k} / sqrt(N_t), theta = e^{+2 pi i/N_t}."""
    jk = np.outer(np.arange(Nt), np.arange(Nt))
    return np.exp(2j * np.pi * jk / Nt) / np.sqrt(Nt)


def preconditioner_dense(A: np.ndarray, tau: float, Nt: int, eps: float) -> np.ndarray:
    """P_eps = C_eps kron I_s - tau I_t kron A (eq. (3.1))."""
    M = A.shape[0]
    return np.kron(C_eps_dense(Nt, eps), np.eye(M)) - tau * np.kron(np.eye(Nt), A)


def pinv_dense(v: np.ndarray, A: np.ndarray, tau: float, eps: float) -> np.ndarray:
    """P_eps^{-1} v by a dense solve (tiny sizes); v has shape [N_t][M]."""
    Nt, M = v.shape
    return np.linalg.solve(preconditioner_dense(A, tau, Nt, eps), v.ravel()).reshape(Nt, M)


def n_unique(Nt: int) -> int:
    """Number of shifted systems that must be solved: floor(N_t/2) + 1.

    Section 3.2 shows z2_{N_t-n} = conj(z2_n) (0-based n); n = 0 and, for even N_t,
    n = N_t/2 are their own partners, so floor(N_t/2)+1 systems remain (the printed
    count floor((N_t+1)/2) omits one of them when N_t is even)."""
    return Nt // 2 + 1


def _along_time(s: np.ndarray, ndim: int) -> np.ndarray:
    """Reshape a per-time-level factor so it broadcasts over [N_t][...]."""
    return s.reshape((-1,) + (1,) * (ndim - 1))


def step_a(v: np.ndarray, eps: float) -> np.ndarray:
    """Step (a): z1_n = sum_j theta^{n j} s_j v_j for n = 0..floor(N_t/2) (half spectrum)."""
    Nt = v.shape[0]
    w = _along_time(scaling_s(Nt, eps), v.ndim) * v
    z1 = Nt * sfft.ifft(w, axis=0)
    return z1[: n_unique(Nt)]


def shifted_matrix(lam: complex, A: np.ndarray, tau: float) -> np.ndarray:
    """B_n = lambda_n I - tau A (Step (b), eq. (3.5))."""
    return lam * np.eye(A.shape[0]) - tau * A


def step_b_exact(z1: np.ndarray, A: np.ndarray, tau: float, Nt: int, eps: float,
                 ns=None) -> np.ndarray:
    """Step (b): z2_n = B_n^{-1} z1_n by LU with partial pivoting (scipy).

    z1 holds the half spectrum (row n = frequency n).  With ns given, only those
    frequencies are solved and the rows are returned in the order of ns."""
    lam = eigenvalues(Nt, eps)
    ns = list(range(z1.shape[0])) if ns is None else list(ns)
    out = np.empty((len(ns), z1.shape[1]), dtype=np.complex128)
    for row, n in enumerate(ns):
        lu = sla.lu_factor(shifted_matrix(lam[n], A, tau))
        out[row] = sla.lu_solve(lu, z1[n])
    return out


def step_c(z2_half: np.ndarray, Nt: int, eps: float) -> np.ndarray:
    """Step (c): extend by z2_{N_t-n} = conj(z2_n), then v_j = s_j^{-1} (1/N_t)
    sum_n theta^{-n j} z2_n.  The result is real; its imaginary part is dropped."""
    full = np.empty((Nt,) + z2_half.shape[1:], dtype=np.complex128)
    nh = n_unique(Nt)
    full[:nh] = z2_half
    for n in range(nh, Nt):
        full[n] = np.conj(z2_half[Nt - n])
    v = sfft.fft(full, axis=0) / Nt
    return (v / _along_time(scaling_s(Nt, eps), v.ndim)).real


def step_c_complex(z2_half: np.ndarray, Nt: int, eps: float) -> np.ndarray:
    """Step (c) without dropping the imaginary part (used to check it vanishes)."""
    full = np.empty((Nt,) + z2_half.shape[1:], dtype=np.complex128)
    nh = n_unique(Nt)
    full[:nh] = z2_half
    for n in range(nh, Nt):
        full[n] = np.conj(z2_half[Nt - n])
    return sfft.fft(full, axis=0) / Nt / _along_time(scaling_s(Nt, eps), full.ndim)


def pinv_fast(v: np.ndarray, A: np.ndarray, tau: float, eps: float) -> np.ndarray:
    """P_eps^{-1} v by steps (a)-(c) of Section 3.1 with exact shifted solves."""
    Nt = v.shape[0]
    z1 = step_a(v, eps)
    z2 = step_b_exact(z1, A, tau, Nt, eps)
    return step_c(z2, Nt, eps)


# ---------------------------------------------------------------------------------
# tau-matrix (DST-I) approximation of the Toeplitz block, eq. (3.9)-(3.11)

def dst_matrix(n: int) -> np.ndarray:
    """Q_n[i, j] = sqrt(2/(n+1)) sin(pi i j / (n+1)), 1 <= i, j <= n (eq. (3.9)).
    Q is symmetric and orthogonal (Q Q = I)."""
    ij = np.outer(np.arange(1, n + 1), np.arange(1, n + 1))
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.pi * ij / (n + 1))


def tau_first_column(t: np.ndarray) -> np.ndarray:
    """First column of the natural tau approximation of a symmetric Toeplitz matrix with
    first column t: t_k - t_{k+2} for k = 0..n-3, the last two entries unchanged.

    Reading of eq. (3.10): the sigma formula needs the first column of the tau matrix
    (Hankel correction removed), not of the Toeplitz matrix itself; the literal reading
    does not reproduce the iteration counts of Tables 1-3."""
    n = len(t)
    c = np.array(t, dtype=np.float64, copy=True)
    if n >= 3:
        c[: n - 2] = t[: n - 2] - t[2:]
    return c


def tau_eigenvalues(t: np.ndarray) -> np.ndarray:
    """sigma_i = (Q chat)_i / Q_{i,1} (eq. (3.10)) with chat = tau_first_column(t)."""
    n = len(t)
    Q = dst_matrix(n)
    return (Q @ tau_first_column(t)) / Q[:, 0]


def tau_matrix(t: np.ndarray) -> np.ndarray:
    """Dense tau matrix Q diag(sigma) Q."""
    Q = dst_matrix(len(t))
    return Q @ np.diag(tau_eigenvalues(t)) @ Q


def step_b_tau(z1: np.ndarray, sigma_A: np.ndarray, tau: float, Nt: int, eps: float) -> np.ndarray:
    """Step (b) with A replaced by its tau approximation Q diag(sigma_A) Q (eq. (3.11)):
    z2_n = Q diag(1/(lambda_n - tau sigma_A)) Q z1_n, for the half spectrum."""
    lam = eigenvalues(Nt, eps)[: z1.shape[0]]
    Q = dst_matrix(z1.shape[1])
    y = z1 @ Q.T
    y = y / (lam[:, None] - tau * sigma_A[None, :])
    return y @ Q.T


def pinv_tau(v: np.ndarray, sigma_A: np.ndarray, tau: float, eps: float) -> np.ndarray:
    """P^{-1} v with the tau/DST step (b) (the paper's own implementation, eq. (3.11))."""
    Nt = v.shape[0]
    return step_c(step_b_tau(step_a(v, eps), sigma_A, tau, Nt, eps), Nt, eps)
