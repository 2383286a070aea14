"""Pins for the FP64 reference of the learned-guess network: chain-rule gradients against central
finite differences, Adam against its closed form on a quadratic, and the sine projection /
synthesis pair against the orthogonality of the DST-I vectors."""
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
