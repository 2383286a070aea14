"""Plain FP64 reference of the learned initial-guess network (test infrastructure only).

The network maps the problem parameters to the responses of the all-at-once solution to each
of the 16 sine-mode data components, in the first Ks sine modes of x:

  features p (B x P_in), standardised: phat = (p - mu) / sd
  h1 = tanh(phat W1^T + b1)                  W1: H1 x P_in
  h2 = tanh(h1 W2^T + b2)                    W2: H2 x H1
  g  = h2 W3t^T + b3                          W3t: NOUT x H2,  NOUT = nsrc * Nt * Ks
  loss = mean over B x NOUT of (g - y)^2

Because the solution of the linear all-at-once system (eq. (2.11)) is linear in the data, the
initial guess for data coefficients c_k is U = sum_k c_k scale_k G_k with G_k the k-th block of g,
synthesised in space as U[t][i] = sum_s Y[t][s] sin(s pi x_i).

Adam (Kingma and Ba, 2015): m = b1 m + (1-b1) grad, v = b2 v + (1-b2) grad^2,
w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np


def forward(params, p, mu, sd):
    W1, b1, W2, b2, W3t, b3 = params
    phat = (p - mu) / sd
    h1 = np.tanh(phat @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    g = h2 @ W3t.T + b3
    return phat, h1, h2, g


def loss(params, p, y, mu, sd):
    g = forward(params, p, mu, sd)[3]
    return float(np.mean((g - y) ** 2))


def grads(params, p, y, mu, sd):
    """Gradients of loss() with respect to (W1, b1, W2, b2, W3t, b3) by the chain rule."""
    W1, b1, W2, b2, W3t, b3 = params
    phat, h1, h2, g = forward(params, p, mu, sd)
    B, NOUT = g.shape
    dg = 2.0 * (g - y) / (B * NOUT)
    dW3t = dg.T @ h2
    db3 = dg.sum(axis=0)
    dh2 = dg @ W3t
    da2 = dh2 * (1.0 - h2**2)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (1.0 - h1**2)
    dW1 = da1.T @ phat
    db1 = da1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3t, db3]


def adam_step(w, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad**2
    mhat = m / (1.0 - b1**t)
    vhat = v / (1.0 - b2**t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v


def sine_basis(M: int, Ks: int) -> np.ndarray:
    """S[i][s] = sin((s+1) pi x_i), x_i = (i+1)/(M+1): the DST-I vectors of the interior grid."""
    i = np.arange(1, M + 1)[:, None]
    s = np.arange(1, Ks + 1)[None, :]
    return np.sin(np.pi * i * s / (M + 1))


def project(U: np.ndarray, Ks: int) -> np.ndarray:
    """Y[t][s] = (2/(M+1)) sum_i U[t][i] sin((s+1) pi x_i): coefficients in the first Ks modes
    (the DST-I vectors are orthogonal with squared norm (M+1)/2)."""
    M = U.shape[-1]
    return U @ sine_basis(M, Ks) * (2.0 / (M + 1))


def synthesize(Y: np.ndarray, M: int) -> np.ndarray:
    """U[t][i] = sum_s Y[t][s] sin((s+1) pi x_i)."""
    return Y @ sine_basis(M, Y.shape[-1]).T


def guess(g_row: np.ndarray, coef: np.ndarray, scale: np.ndarray, Nt: int, Ks: int, M: int):
    """U_guess = synthesize(sum_k coef_k scale_k G_k) for one network output row g_row."""
    G = g_row.reshape(len(coef), Nt, Ks)
    Y = np.tensordot(coef * scale, G, axes=(0, 0))
    return synthesize(Y, M)
