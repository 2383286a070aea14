"""Two-dimensional model (Section 4, eq. (4.1)-(4.5)).

Layout: a spatial field is u[iy][ix] with x fastest (flat index iy*Mx + ix); a space-time
vector is [N_t][My][Mx].  The Jacobian of eq. (4.2) is the Kronecker sum
A = -(c_x T_x (on the x index) + c_y T_y (on the y index)), c = kappa / h^gamma; in the
x-fastest layout this is -(c_x kron(I_y, T_x) + c_y kron(T_y, I_x)).
"""
from __future__ import annotations

import numpy as np

from .allatonce import toeplitz_T
from .precond import (dst_matrix, eigenvalues, n_unique, step_a, step_c,
                      tau_eigenvalues)
from .weights import gk_recurrence


def coeffs(gx, gy, kx, ky, hx, hy):
    """c_x = kappa_x / h_x^{gamma_x}, c_y = kappa_y / h_y^{gamma_y} (eq. (4.2))."""
    return kx / hx**gx, ky / hy**gy


def jacobian_2d_dense(gx, gy, kx, ky, hx, hy, Mx, My) -> np.ndarray:
    """Dense A of eq. (4.2) in the x-fastest layout (tiny grids only)."""
    cx, cy = coeffs(gx, gy, kx, ky, hx, hy)
    return -(cx * np.kron(np.eye(My), toeplitz_T(gx, Mx))
             + cy * np.kron(toeplitz_T(gy, My), np.eye(Mx)))


def apply_spatial(u: np.ndarray, Tx: np.ndarray, Ty: np.ndarray, cx: float, cy: float) -> np.ndarray:
    """A u for u[..., My, Mx]: -(c_x u T_x^T along x + c_y T_y u along y)."""
    return -(cx * (u @ Tx.T) + cy * np.einsum("yk,...kx->...yx", Ty, u))


def apply_all_at_once_2d(v: np.ndarray, Tx, Ty, cx, cy, tau) -> np.ndarray:
    """(C kron I - tau I kron A) v for v[N_t][My][Mx] (eq. (2.11) with the 2D A)."""
    Nt = v.shape[0]
    y = np.empty_like(v)
    y[0] = v[0]
    if Nt > 1:
        y[1] = 1.5 * v[1] - 2.0 * v[0]
    for k in range(2, Nt):
        y[k] = 1.5 * v[k] - 2.0 * v[k - 1] + 0.5 * v[k - 2]
    return y - tau * apply_spatial(v, Tx, Ty, cx, cy)


class ShiftedSolver2D:
    """Direct solver for (s I - tau A) u = r by fast diagonalization (Lynch-Rice-Thomas):
    T_x = Qx diag(mx) Qx^T, T_y = Qy diag(my) Qy^T (symmetric eigensolver), so
    s I - tau A = (Qy kron Qx) diag(s + tau (c_x mx_i + c_y my_j)) (Qy kron Qx)^T."""

    def __init__(self, Tx, Ty, cx, cy, tau):
        self.mx, self.Qx = np.linalg.eigh(Tx)
        self.my, self.Qy = np.linalg.eigh(Ty)
        self.d = tau * (cy * self.my[:, None] + cx * self.mx[None, :])

    def solve(self, s, r):
        t = self.Qy.T @ r @ self.Qx
        t = t / (s + self.d)
        return self.Qy @ t @ self.Qx.T


def bdf2_march_2d(u0, f, Tx, Ty, cx, cy, tau) -> np.ndarray:
    """U* of the 2D all-at-once system by marching eq. (1.2a)-(1.2b) level by level."""
    S = ShiftedSolver2D(Tx, Ty, cx, cy, tau)
    Nt = f.shape[0]
    U = np.empty_like(f)
    U[0] = S.solve(1.0, tau * f[0] + u0)
    for k in range(1, Nt):
        prev2 = u0 if k == 1 else U[k - 2]
        U[k] = S.solve(1.5, tau * f[k] + 2.0 * U[k - 1] - 0.5 * prev2)
    return U


def tau_sigma_2d(gx, gy, Mx, My):
    """Eigenvalues of the tau approximations of T_x and T_y (eq. (4.4))."""
    return tau_eigenvalues(gk_recurrence(gx, Mx)), tau_eigenvalues(gk_recurrence(gy, My))


def step_b_tau_2d(z1, sx, sy, cx, cy, tau, Nt, eps):
    """Step (b) with the 2D tau approximation (eq. (4.5), read as
    [lambda_n I + tau (c_x Lambda^x (+) c_y Lambda^y)] in the (Qy kron Qx) basis):
    z2_n = (Qy kron Qx) diag(1 / (lambda_n + tau (c_x sx_i + c_y sy_j))) (Qy kron Qx) z1_n."""
    lam = eigenvalues(Nt, eps)[: z1.shape[0]]
    My, Mx = z1.shape[1], z1.shape[2]
    Qx, Qy = dst_matrix(Mx), dst_matrix(My)
    t = np.einsum("yk,nkx->nyx", Qy, z1 @ Qx)
    t = t / (lam[:, None, None] + tau * (cy * sy[None, :, None] + cx * sx[None, None, :]))
    return np.einsum("yk,nkx->nyx", Qy, t @ Qx)


def pinv_tau_2d(v, sx, sy, cx, cy, tau, eps):
    """P^{-1} v for v[N_t][My][Mx] with the 2D tau/DST shifted solves."""
    Nt = v.shape[0]
    return step_c(step_b_tau_2d(step_a(v, eps), sx, sy, cx, cy, tau, Nt, eps), Nt, eps)


def step_b_exact_2d(z1, Tx, Ty, cx, cy, tau, Nt, eps, ns=None):
    """Step (b) with the exact 2D shifted operator B_n = lambda_n I - tau A, by fast
    diagonalization; rows follow ns (default: the half spectrum)."""
    lam = eigenvalues(Nt, eps)
    S = ShiftedSolver2D(Tx, Ty, cx, cy, tau)
    ns = list(range(z1.shape[0])) if ns is None else list(ns)
    return np.array([S.solve(lam[n], z1[n]) for n in ns])


def step_b_inner_2d(z1, Tx, Ty, sx, sy, cx, cy, tau, Nt, eps, k, inner_tol=0.0, ns=None):
    """Step (b) with an inner solver on the exact shifted operator (the optional inner
    iteration of the 2D step (b), the paper giving only the tau approximation of eq. (4.5)):
    for each frequency n, GMRES on B_n x = z1_n with B_n = lambda_n I - tau A, zero start,
    right-preconditioned by that frequency's tau solve, at most k steps.  Textbook GMRES:
    Arnoldi with modified Gram-Schmidt and Hermitian inner products on B_n P_n^{-1}, the small
    least-squares problem min ||beta e_1 - H y|| solved directly, x = P_n^{-1} V y.  With
    inner_tol > 0 every frequency stops after the first step at which all of them have
    ||z1_n - B_n x_n|| <= inner_tol ||z1_n||.  Rows follow ns (default: the half spectrum).
    Returns (x, steps taken)."""
    nfq, My, Mx = z1.shape
    ns = list(range(nfq)) if ns is None else list(ns)
    lam = eigenvalues(Nt, eps)[ns]
    Qx, Qy = dst_matrix(Mx), dst_matrix(My)
    den = tau * (cy * sy[:, None] + cx * sx[None, :])

    def prec(n, r):
        return Qy @ ((Qy @ r @ Qx) / (lam[n] + den)) @ Qx

    def op(n, z):
        return lam[n] * z - tau * apply_spatial(z, Tx, Ty, cx, cy)

    beta = np.array([np.linalg.norm(z1[n]) for n in range(nfq)])
    V = [[z1[n] / beta[n] if beta[n] > 0 else np.zeros_like(z1[n])] for n in range(nfq)]
    Z = [[] for _ in range(nfq)]
    H = np.zeros((nfq, k + 1, k), dtype=np.complex128)

    def lsq(n, m):
        rhs = np.zeros(m + 1, dtype=np.complex128)
        rhs[0] = beta[n]
        y = np.linalg.lstsq(H[n, : m + 1, :m], rhs, rcond=None)[0]
        return y, np.linalg.norm(rhs - H[n, : m + 1, :m] @ y)

    steps = k
    for j in range(k):
        for n in range(nfq):
            z = prec(n, V[n][j])
            Z[n].append(z)
            w = op(n, z)
            for i in range(j + 1):
                H[n, i, j] = np.vdot(V[n][i], w)
                w = w - H[n, i, j] * V[n][i]
            H[n, j + 1, j] = np.linalg.norm(w)
            V[n].append(w / H[n, j + 1, j] if H[n, j + 1, j] > 0 else np.zeros_like(w))
        if inner_tol > 0 and all(lsq(n, j + 1)[1] <= inner_tol * beta[n] for n in range(nfq)):
            steps = j + 1
            break
    x = np.zeros_like(z1, dtype=np.complex128)
    for n in range(nfq):
        if beta[n] > 0 and steps > 0:
            y = lsq(n, steps)[0]
            x[n] = sum(y[i] * Z[n][i] for i in range(steps))
    return x, steps


__all__ = ["coeffs", "jacobian_2d_dense", "apply_spatial", "apply_all_at_once_2d",
           "ShiftedSolver2D", "bdf2_march_2d", "tau_sigma_2d", "step_b_tau_2d",
           "pinv_tau_2d", "step_b_exact_2d", "step_b_inner_2d", "n_unique"]
