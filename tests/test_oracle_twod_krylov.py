"""Pins for the 2D oracle (eq. (4.1)-(4.5)) and the FGMRES oracle."""
import numpy as np
import pytest

from oracle import allatonce as aa
from oracle import krylov
from oracle import precond as pc
from oracle import twod
from rfde_workloads import gen2d


def _setup2d(gx=1.6, gy=1.4, Mx=6, My=5, Nt=6):
    hx, hy = 1.0 / (Mx + 1), 1.0 / (My + 1)
    tau = 1.0 / Nt
    Tx, Ty = aa.toeplitz_T(gx, Mx), aa.toeplitz_T(gy, My)
    cx, cy = twod.coeffs(gx, gy, 1.0, 1.0, hx, hy)
    return hx, hy, tau, Tx, Ty, cx, cy


def test_spatial_operator_matches_dense_kronecker():
    hx, hy, tau, Tx, Ty, cx, cy = _setup2d()
    A = twod.jacobian_2d_dense(1.6, 1.4, 1.0, 1.0, hx, hy, 6, 5)
    u = np.random.default_rng(0).standard_normal((5, 6))
    assert np.allclose(twod.apply_spatial(u, Tx, Ty, cx, cy).ravel(), A @ u.ravel(), atol=1e-12)
    # A is negative definite (SPD up to sign)
    assert np.linalg.eigvalsh(A).max() < 0


def test_x_y_roles_swap():
    # transposing the grid swaps the roles of (gamma_x, h_x) and (gamma_y, h_y)
    hx, hy, tau, Tx, Ty, cx, cy = _setup2d()
    u = np.random.default_rng(1).standard_normal((5, 6))
    a = twod.apply_spatial(u, Tx, Ty, cx, cy)
    b = twod.apply_spatial(u.T, Ty, Tx, cy, cx)
    assert np.allclose(a, b.T, atol=1e-13)


def test_march_2d_equals_dense_solve():
    hx, hy, tau, Tx, Ty, cx, cy = _setup2d()
    Nt = 6
    u0, f, _ = gen2d(3, 6, 5, Nt)
    U = twod.bdf2_march_2d(u0, f, Tx, Ty, cx, cy, tau)
    A = twod.jacobian_2d_dense(1.6, 1.4, 1.0, 1.0, hx, hy, 6, 5)
    Ud = aa.dense_direct(u0.ravel(), f.reshape(Nt, -1), A, tau).reshape(U.shape)
    assert np.max(np.abs(U - Ud)) < 1e-12 * np.max(np.abs(Ud))
    # and the all-at-once 2D matvec of U reproduces F
    y = twod.apply_all_at_once_2d(U, Tx, Ty, cx, cy, tau)
    F = aa.rhs_F(u0, f, tau)
    assert np.max(np.abs(y - F)) < 1e-12 * np.max(np.abs(F))


def test_tau_preconditioner_2d_matches_dense():
    gx, gy, Mx, My, Nt = 1.6, 1.4, 6, 5, 6
    hx, hy, tau, Tx, Ty, cx, cy = _setup2d(gx, gy, Mx, My, Nt)
    eps = pc.default_eps(tau)
    sx, sy = twod.tau_sigma_2d(gx, gy, Mx, My)
    Atau = -(cx * np.kron(np.eye(My), pc.tau_matrix(aa.toeplitz_T(gx, Mx)[:, 0]))
             + cy * np.kron(pc.tau_matrix(aa.toeplitz_T(gy, My)[:, 0]), np.eye(Mx)))
    P = pc.preconditioner_dense(Atau, tau, Nt, eps)
    v = np.random.default_rng(4).standard_normal((Nt, My, Mx))
    zd = np.linalg.solve(P, v.ravel()).reshape(v.shape)
    zf = twod.pinv_tau_2d(v, sx, sy, cx, cy, tau, eps)
    assert np.max(np.abs(zf - zd)) < 1e-12 * np.max(np.abs(zd))
    # exact shifted operator via fast diagonalization vs dense B_n
    A = twod.jacobian_2d_dense(gx, gy, 1.0, 1.0, hx, hy, Mx, My)
    z1 = pc.step_a(v.reshape(Nt, -1), eps).reshape(-1, My, Mx)
    z2 = twod.step_b_exact_2d(z1, Tx, Ty, cx, cy, tau, Nt, eps)
    lam = pc.eigenvalues(Nt, eps)
    for n in range(z1.shape[0]):
        ref = np.linalg.solve(pc.shifted_matrix(lam[n], A, tau), z1[n].ravel())
        assert np.allclose(z2[n].ravel(), ref, atol=1e-12 * np.abs(ref).max())


def test_fgmres_solves_small_system_and_terminates():
    rng = np.random.default_rng(5)
    n = 12
    A = np.eye(n) * 4 + rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    x, info = krylov.fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-12, restart=n)
    assert info["converged"] and info["iters"] <= n
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-10)
    # with a restart shorter than n it still converges (restart path)
    x2, info2 = krylov.fgmres(lambda v: A @ v, lambda v: v, b, tol=1e-10, restart=4, maxit=400)
    assert info2["converged"]
    assert np.allclose(x2, np.linalg.solve(A, b), atol=1e-8)


def test_fgmres_iterations_bounded_by_rank():
    # Theorem 3.1 (corrected rank 2 N_s): right-preconditioned GMRES with P_eps terminates
    # in at most 2 N_s + 1 iterations in exact arithmetic; check it on a small case
    gam, Nt, M = 1.5, 12, 4
    h, tau = aa.mesh(0, 1, M, 1.0, Nt)
    A = aa.jacobian_A(gam, 1.0, h, M)
    eps = pc.default_eps(tau)
    b = np.random.default_rng(6).standard_normal(Nt * M)
    Av = lambda v: aa.apply_all_at_once(v.reshape(Nt, M), A, tau).ravel()
    Mv = lambda v: pc.pinv_dense(v.reshape(Nt, M), A, tau, eps).ravel()
    x, info = krylov.fgmres(Av, Mv, b, tol=1e-11)
    assert info["iters"] <= 2 * M + 1
    assert info["true_rel_res"] <= 1e-11
