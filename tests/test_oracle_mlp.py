"""Pins for the FP64 reference of the learned-guess network: chain-rule gradients against central
finite differences, Adam against its closed form on a quadratic, and the sine projection /
synthesis pair against the orthogonality of the DST-I vectors, and the guess assembly against a
hand-built case and against the projection of oracle solutions (linearity of eq. (2.11))."""
import math

import numpy as np
import pytest

from oracle import mlp


def _params(rng, Pin=3, H1=5, H2=6, NOUT=7):
    return [rng.standard_normal((H1, Pin)) * 0.5, rng.standard_normal(H1) * 0.1,
            rng.standard_normal((H2, H1)) * 0.5, rng.standard_normal(H2) * 0.1,
            rng.standard_normal((NOUT, H2)) * 0.5, rng.standard_normal(NOUT) * 0.1]


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    params = _params(rng)
    B = 4
    p = rng.standard_normal((B, 3))
    y = rng.standard_normal((B, 7))
    mu, sd = np.array([0.1, -0.2, 0.3]), np.array([1.5, 0.7, 2.0])
    g = mlp.grads(params, p, y, mu, sd)
    h = 1e-6
    for a, P in enumerate(params):
        for idx in np.ndindex(P.shape):
            old = P[idx]
            P[idx] = old + h
            lp = mlp.loss(params, p, y, mu, sd)
            P[idx] = old - h
            lm = mlp.loss(params, p, y, mu, sd)
            P[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[a][idx]) <= 1e-7 * max(1.0, abs(fd)), (a, idx)


def test_adam_minimises_quadratic_and_first_step():
    # first step from m = v = 0 moves every coordinate by lr * sign(grad) (up to eps)
    w = np.array([1.0, -2.0, 3.0])
    grad = np.array([0.5, -4.0, 1e-3])
    w1, m, v = mlp.adam_step(w, grad, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(w1, w - 0.01 * np.sign(grad), atol=1e-7)
    # and it converges on a convex quadratic
    w = np.array([3.0, -1.0])
    m = v = np.zeros(2)
    for t in range(1, 3001):
        w, m, v = mlp.adam_step(w, 2 * (w - np.array([0.5, 0.25])), m, v, t, lr=0.01)
    assert np.allclose(w, [0.5, 0.25], atol=1e-3)


@pytest.mark.parametrize("M,Ks", [(15, 4), (63, 16), (1023, 64)])
def test_project_synthesize_roundtrip(M, Ks):
    rng = np.random.default_rng(M)
    Y = rng.standard_normal((5, Ks))
    assert np.allclose(mlp.project(mlp.synthesize(Y, M), Ks), Y, atol=1e-12)
    S = mlp.sine_basis(M, Ks)
    assert np.allclose(S.T @ S, np.eye(Ks) * (M + 1) / 2, atol=1e-9)


def test_guess_hand_built_case():
    # nsrc = 2 components, N_t = 3 levels, Ks = 4 modes, M = 5 points: every entry of the
    # network row is distinct, so any transposition of the (component, level, mode) axes or of
    # the (level, point) output changes the result
    nsrc, Nt, Ks, M = 2, 3, 4, 5
    g_row = np.arange(1.0, nsrc * Nt * Ks + 1.0)
    coef = np.array([2.0, -1.0])
    scale = np.array([0.5, 3.0])
    want = np.zeros((Nt, M))
    for t in range(Nt):
        for i in range(M):
            acc = 0.0
            for k in range(nsrc):
                for s in range(Ks):
                    acc += coef[k] * scale[k] * g_row[k * Nt * Ks + t * Ks + s] \
                        * math.sin((s + 1) * math.pi * (i + 1) / (M + 1))
            want[t, i] = acc
    got = mlp.guess(g_row, coef, scale, Nt, Ks, M)
    assert got.shape == (Nt, M)
    assert np.allclose(got, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("Ks", [15, 6])
def test_guess_from_unit_solutions_is_projected_solution(Ks):
    # eq. (2.11): F is linear in (u0, f), so for fixed (alpha, kappa) the all-at-once solution
    # for data sum_j c_j (unit component j) is sum_j c_j G_j.  Filling the network row with the
    # projected unit solutions must give the projection of the combined solution, which for
    # Ks = M (a complete sine basis) is the solution itself.
    import rfde_workloads as wl
    from oracle import allatonce as aa
    M, Nt, T, alpha, kappa = 15, 8, 1.0, 1.6, 0.7
    h, tau = aa.mesh(0.0, 1.0, M, T, Nt)
    A = aa.jacobian_A(alpha, kappa, h, M)
    rows = []
    for j in range(16):
        u0j, fj = wl.unit_data(j, M, Nt, T)
        rows.append(mlp.project(aa.bdf2_march(u0j, fj, A, tau), Ks))
    g_row = np.stack(rows).ravel()                      # layout [component][level][mode]
    u0, f, (ak, bk) = wl.gen1d(77, M, Nt, T)
    coef = np.concatenate([ak, bk])
    U = aa.bdf2_march(u0, f, A, tau)
    got = mlp.guess(g_row, coef, np.ones(16), Nt, Ks, M)
    want = mlp.synthesize(mlp.project(U, Ks), M)
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(U))
    if Ks == M:
        assert np.max(np.abs(got - U)) < 1e-12 * np.max(np.abs(U))
    # linearity in the coefficients
    c2 = np.random.default_rng(3).standard_normal(16)
    lin = mlp.guess(g_row, coef + 2.0 * c2, np.ones(16), Nt, Ks, M)
    assert np.allclose(lin, got + 2.0 * mlp.guess(g_row, c2, np.ones(16), Nt, Ks, M),
                       rtol=0, atol=1e-12 * np.max(np.abs(lin)))
