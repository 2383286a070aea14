"""Spatial Toeplitz block, BDF2 scheme and the all-at-once system (Section 2).

Vector layout: U = (u^1; u^2; ...; u^{N_t}) stacked in time, each u^k of length M
(the paper's N_s = N - 1), so the flat index is k*M + i (eq. (2.11)).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .weights import gk_recurrence


def mesh(a: float, b: float, M: int, T: float, Nt: int):
    """h = (b - a)/(M + 1) and tau = T / N_t (Section 2.1, M interior points)."""
    return (b - a) / (M + 1), T / Nt


def toeplitz_T(gam: float, M: int) -> np.ndarray:
    """Dense T_x (eq. (2.9)): T[i, j] = omega_{|i-j|}, symmetric Toeplitz of order M."""
    return sla.toeplitz(gk_recurrence(gam, M))


def jacobian_A(gam: float, kappa: float, h: float, M: int) -> np.ndarray:
    """A = -kappa h^{-gam} T_x (eq. (2.9)), the discrete kappa * Riesz derivative."""
    return -(kappa / h**gam) * toeplitz_T(gam, M)


def time_matrix_C(Nt: int) -> np.ndarray:
    """C of eq. (2.12): rows (1); (-2, 3/2); (1/2, -2, 3/2) shifted down the diagonal.

    The BDF2 stencil is (3u^k - 4u^{k-1} + u^{k-2}) / (2 tau) as in eq. (1.2b); the
    coefficients printed in eq. (2.6)-(2.7) have the first and last swapped, and the
    matrix C (and the error values of the examples) fix the reading used here.
    """
    C = np.zeros((Nt, Nt))
    C[0, 0] = 1.0
    for k in range(1, Nt):
        C[k, k] = 1.5
        C[k, k - 1] = -2.0
        if k >= 2:
            C[k, k - 2] = 0.5
    return C


def all_at_once_matrix(C: np.ndarray, A: np.ndarray, tau: float) -> np.ndarray:
    """Dense all-at-once matrix = C kron I_s - tau I_t kron A (eq. (2.11)-(2.12))."""
    Nt, M = C.shape[0], A.shape[0]
    return np.kron(C, np.eye(M)) - tau * np.kron(np.eye(Nt), A)


def rhs_F(u0: np.ndarray, f: np.ndarray, tau: float) -> np.ndarray:
    """Right-hand side of eq. (2.11): F_1 = tau f^1 + u^0, F_2 = tau f^2 - u^0/2,
    F_k = tau f^k otherwise.  f has shape [N_t][...] holding f^1..f^{N_t}."""
    F = tau * np.array(f, dtype=np.float64, copy=True)
    F[0] += u0
    if F.shape[0] > 1:
        F[1] -= 0.5 * u0
    return F


def apply_all_at_once(v: np.ndarray, A: np.ndarray, tau: float) -> np.ndarray:
    """(C kron I - tau I kron A) v for v of shape [N_t][M], written as
    vec(V C^T) - tau vec(A V) (Section 3.2), with A applied densely per time level."""
    Nt = v.shape[0]
    y = np.empty_like(v)
    for k in range(Nt):
        if k == 0:
            y[k] = v[0]
        elif k == 1:
            y[k] = 1.5 * v[1] - 2.0 * v[0]
        else:
            y[k] = 1.5 * v[k] - 2.0 * v[k - 1] + 0.5 * v[k - 2]
    y -= tau * (v @ A.T)
    return y


def bdf2_march(u0: np.ndarray, f: np.ndarray, A: np.ndarray, tau: float) -> np.ndarray:
    """U* by time marching eq. (1.2a)-(1.2b), one level after the other.

    (I - tau A) u^1 = tau f^1 + u^0,
    (3/2 I - tau A) u^k = tau f^k + 2 u^{k-1} - 1/2 u^{k-2}   (k >= 2).
    Both matrices are SPD (A is negative definite), so each uses a Cholesky factor.
    Because C is lower triangular this is exactly the solution of eq. (2.11).
    Returns U of shape [N_t][M].
    """
    Nt, M = f.shape
    I = np.eye(M)
    c1 = sla.cho_factor(I - tau * A)
    c2 = sla.cho_factor(1.5 * I - tau * A) if Nt > 1 else None
    U = np.empty((Nt, M))
    U[0] = sla.cho_solve(c1, tau * f[0] + u0)
    for k in range(1, Nt):
        prev2 = u0 if k == 1 else U[k - 2]
        U[k] = sla.cho_solve(c2, tau * f[k] + 2.0 * U[k - 1] - 0.5 * prev2)
    return U


def bdf2_march_eig(u0: np.ndarray, f: np.ndarray, A: np.ndarray, tau: float) -> np.ndarray:
    """The same march as bdf2_march, with A = Q diag(mu) Q^T (symmetric eigensolver).

    In the eigenbasis each BDF2 step is a scalar recursion per mode, so all N_t levels
    cost two matrix products.  Used at sizes where N_t dense triangular solves are slow.
    """
    mu, Q = np.linalg.eigh(A)
    fh = (tau * f) @ Q                   # rows are Q^T (tau f^k)
    uh0 = u0 @ Q
    Nt = f.shape[0]
    Uh = np.empty_like(fh)
    Uh[0] = (fh[0] + uh0) / (1.0 - tau * mu)
    d2 = 1.5 - tau * mu
    for k in range(1, Nt):
        prev2 = uh0 if k == 1 else Uh[k - 2]
        Uh[k] = (fh[k] + 2.0 * Uh[k - 1] - 0.5 * prev2) / d2
    return Uh @ Q.T


def dense_direct(u0: np.ndarray, f: np.ndarray, A: np.ndarray, tau: float) -> np.ndarray:
    """U = (all-at-once matrix)^{-1} F by a dense LU solve (tiny sizes only)."""
    Nt, M = f.shape
    Aall = all_at_once_matrix(time_matrix_C(Nt), A, tau)
    return np.linalg.solve(Aall, rhs_F(u0, f, tau).ravel()).reshape(Nt, M)


def C_inverse_closed_form(Nt: int) -> np.ndarray:
    """Lemma 2.3: C^{-1} = Chat^{-1} + (1/2) w e_1^T with Chat^{-1}[i, j] = 1 - 3^{-(i-j+1)}
    for i >= j, and w = Chat^{-1} e_1, w_i = 1 - 3^{-(i+1)} (0-based i)."""
    i = np.arange(Nt)[:, None]
    j = np.arange(Nt)[None, :]
    Chat_inv = np.where(i >= j, 1.0 - 3.0 ** (-(i - j + 1.0)), 0.0)
    w = 1.0 - 3.0 ** (-(np.arange(Nt) + 1.0))
    out = Chat_inv.copy()
    out[:, 0] += 0.5 * w
    return out


def circulant_symbol(g: np.ndarray, M: int, L: int) -> np.ndarray:
    """Eigenvalues of the symmetric circulant of order L >= 2M-1 whose first column is
    (g_0, ..., g_{M-1}, 0, ..., 0, g_{M-1}, ..., g_1): the DFT of that column (a circulant is
    diagonalised by the Fourier matrix).  T_x is its leading M x M block, which is how the
    Toeplitz product is done in O(L log L) (Section 2.1)."""
    c = np.zeros(L)
    c[:M] = g[:M]
    c[L - M + 1:] = g[1:M][::-1]
    return np.fft.fft(c).real
