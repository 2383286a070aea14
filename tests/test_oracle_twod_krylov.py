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


def _inner_case(Mx=6, My=5, Nt=6, seed=11):
    gx, gy = 1.6, 1.4
    hx, hy, tau, Tx, Ty, cx, cy = _setup2d(gx, gy, Mx, My, Nt)
    eps = pc.default_eps(tau)
    sx, sy = twod.tau_sigma_2d(gx, gy, Mx, My)
    lam = pc.eigenvalues(Nt, eps)
    nf = Nt // 2 + 1
    rng = np.random.default_rng(seed)
    z1 = rng.standard_normal((nf, My, Mx)) + 1j * rng.standard_normal((nf, My, Mx))
    # the two maps written out densely (independent of the oracle's routines): B_n and the
    # tau solve of frequency n as matrices in the x-fastest layout
    Qx, Qy = pc.dst_matrix(Mx), pc.dst_matrix(My)
    Q = np.kron(Qy, Qx)
    A = twod.jacobian_2d_dense(gx, gy, 1.0, 1.0, hx, hy, Mx, My)
    dtau = tau * (cy * np.repeat(sy, Mx) + cx * np.tile(sx, My))
    Bd = [lam[n] * np.eye(Mx * My) - tau * A for n in range(nf)]
    Pd = [Q @ np.diag(1.0 / (lam[n] + dtau)) @ Q for n in range(nf)]
    args = (Tx, Ty, sx, sy, cx, cy, tau, Nt, eps)
    return z1, Bd, Pd, args


def test_inner_one_step_is_the_best_multiple_of_the_tau_solve():
    # k = 1: x = a P^-1 w with a minimising ||w - a B P^-1 w||, a = (u^H w) / (u^H u), u = B P^-1 w
    z1, Bd, Pd, args = _inner_case()
    x, steps = twod.step_b_inner_2d(z1, *args, k=1)
    assert steps == 1
    for n in range(z1.shape[0]):
        w = z1[n].ravel()
        pw = Pd[n] @ w
        u = Bd[n] @ pw
        a = np.vdot(u, w) / np.vdot(u, u)
        assert np.max(np.abs(x[n].ravel() - a * pw)) < 1e-13 * np.max(np.abs(a * pw))


@pytest.mark.parametrize("k", [2, 3])
def test_inner_matches_power_basis_least_squares(k):
    # GMRES(k) from zero with right preconditioner P: x = P K c, K = [w, C w, .., C^{k-1} w],
    # C = B P, c minimising ||w - C K c|| (brute force on the power basis)
    z1, Bd, Pd, args = _inner_case()
    x, steps = twod.step_b_inner_2d(z1, *args, k=k)
    assert steps == k
    for n in range(z1.shape[0]):
        w = z1[n].ravel()
        C = Bd[n] @ Pd[n]
        K = np.stack([np.linalg.matrix_power(C, i) @ w for i in range(k)], axis=1)
        c = np.linalg.lstsq(C @ K, w, rcond=None)[0]
        ref = Pd[n] @ (K @ c)
        assert np.max(np.abs(x[n].ravel() - ref)) < 1e-10 * np.max(np.abs(ref))


def test_inner_reaches_the_exact_solve_and_residuals_do_not_grow():
    # on a 4 x 3 grid, 12 steps span the whole space: x = B^-1 w (fast diagonalisation)
    Mx, My, Nt = 4, 3, 4
    z1, Bd, Pd, args = _inner_case(Mx, My, Nt, seed=12)
    Tx, Ty, sx, sy, cx, cy, tau, Nt, eps = args
    ref = twod.step_b_exact_2d(z1, Tx, Ty, cx, cy, tau, Nt, eps)
    x, _ = twod.step_b_inner_2d(z1, *args, k=Mx * My)
    assert np.max(np.abs(x - ref)) < 1e-10 * np.max(np.abs(ref))
    res = []
    for k in range(1, 6):
        xk, _ = twod.step_b_inner_2d(z1, *args, k=k)
        res.append([np.linalg.norm(z1[n].ravel() - Bd[n] @ xk[n].ravel())
                    for n in range(z1.shape[0])])
    res = np.array(res)
    assert np.all(res[1:] <= res[:-1] * (1 + 1e-12))


def test_inner_tolerance_stops_all_frequencies_together():
    z1, Bd, Pd, args = _inner_case()
    rel = []
    for k in range(1, 7):
        xk, _ = twod.step_b_inner_2d(z1, *args, k=k)
        rel.append(max(np.linalg.norm(z1[n].ravel() - Bd[n] @ xk[n].ravel())
                       / np.linalg.norm(z1[n]) for n in range(z1.shape[0])))
    # a tolerance between the residuals after 2 and 3 steps stops after exactly 3
    tol = np.sqrt(rel[1] * rel[2])
    assert rel[2] < tol < rel[1]
    x, steps = twod.step_b_inner_2d(z1, *args, k=6, inner_tol=tol)
    x3, _ = twod.step_b_inner_2d(z1, *args, k=3)
    assert steps == 3
    assert np.max(np.abs(x - x3)) < 1e-14 * np.max(np.abs(x3))
