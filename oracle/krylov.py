"""Flexible GMRES with right preconditioning (the solver of Section 4).

The paper runs right-preconditioned Ad-SGMRES from the zero vector and stops on
||r_k|| / ||r_0|| < tol.  This oracle is plain restarted FGMRES(m): modified
Gram-Schmidt Arnoldi, Givens rotations, x = x0 + Z y.  For a fixed preconditioner it
produces the same minimal-residual iterates as right-preconditioned GMRES.

Stopping: the Arnoldi residual estimate relative to ||b|| (the true relative residual
TRR of Section 4 when x0 = 0); at each restart and at exit the true residual
||b - A x|| / ||b|| is recomputed, and the solve only ends once it is <= tol.
"""
from __future__ import annotations

import numpy as np


def fgmres(apply_A, apply_M, b: np.ndarray, x0=None, tol: float = 1e-9,
           restart: int = 30, maxit: int = 500):
    """Solve A x = b.  apply_A, apply_M map flat float64 arrays to flat arrays.

    Returns (x, info) with info = dict(iters, converged, true_rel_res, history) where
    history[k] is the estimated ||r_k|| / ||b|| after k Arnoldi steps in total.
    """
    b = np.asarray(b, dtype=np.float64).ravel()
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64).ravel()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros(n), dict(iters=0, converged=True, true_rel_res=0.0, history=[0.0])
    total = 0
    history = []
    r = b - apply_A(x)
    beta = np.linalg.norm(r)
    history.append(beta / bnorm)
    while True:
        if beta / bnorm <= tol or total >= maxit:
            break
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            Z[j] = apply_M(V[j])
            w = apply_A(Z[j])
            for i in range(j + 1):            # modified Gram-Schmidt
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                # apply earlier rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_done = j + 1
            history.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= tol or total >= maxit or H[j, j] == 0.0:
                break
        k = j_done
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):        # back substitution on the triangular H
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + y @ Z[:k]
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol or total >= maxit:
            break
    rel = beta / bnorm
    return x, dict(iters=total, converged=rel <= tol, true_rel_res=rel, history=history)
