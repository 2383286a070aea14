"""Pins for the fractional centred-difference weights (eq. (2.4), Lemma 2.1, Lemma 2.2)."""
import numpy as np
import pytest

from oracle.weights import gk_closed_form, gk_recurrence, gk_tail_sum_asymptote

GAMMAS = (1.1, 1.2, 1.5, 1.8, 1.9)


@pytest.mark.parametrize("gam", GAMMAS)
def test_recurrence_matches_closed_form(gam):
    # eq. (2.4) evaluated directly (log-Gamma with sign) vs the ratio recurrence
    n = 300
    r = gk_recurrence(gam, n)
    c = gk_closed_form(gam, n)
    assert np.max(np.abs(r - c) / np.abs(c)) < 1e-12


@pytest.mark.parametrize("gam", GAMMAS)
def test_signs_and_symmetry(gam):
    # Lemma 2.1: omega_0 >= 0 (here > 0), omega_l < 0 for |l| >= 1, omega_{-l} = omega_l
    g = gk_recurrence(gam, 200)
    assert g[0] > 0
    assert np.all(g[1:] < 0)
    l = np.arange(1, 40, dtype=float)
    from scipy.special import gamma as G, gammaln, gammasgn
    z = 1.0 + gam / 2.0 + l  # argument of Gamma(1 + gam/2 - (-l))
    neg = ((-1.0) ** l) * gammasgn(1 + gam / 2 - l) * np.exp(
        gammaln(1 + gam) - gammaln(z) - gammaln(1 + gam / 2 - l))
    # omega_{-l}: swap the two Gamma factors of eq. (2.4)
    assert np.allclose(neg, g[1:40], rtol=1e-12, atol=0)


@pytest.mark.parametrize("gam", (1.2, 1.5, 1.8))
def test_sum_rule_and_tail(gam):
    # Lemma 2.1: sum over all integers is 0, so S_K = g_0 + 2 sum_{k<=K} g_k > 0 decreases
    # to 0 like the tail asymptote 2 Gamma(1+gam) sin(pi gam/2)/(pi gam) K^-gam
    g = gk_recurrence(gam, 20001)
    S = g[0] + 2.0 * np.cumsum(g[1:])
    assert np.all(S > 0)
    assert np.all(np.diff(S) < 0)
    for K in (1000, 5000, 20000):
        assert abs(S[K - 1] / gk_tail_sum_asymptote(gam, K) - 1.0) < 2e-3 * (1 + 1000 / K)
    # gamma = 1.5, K = 4999 (value independently computed from the asymptote: 1.13e-6)
    if gam == 1.5:
        assert abs(S[4998] - 1.13e-6) < 0.01e-6


def test_gamma_two_is_three_point_laplacian():
    # Lemma 2.2: at gamma = 2 the formula is the second-order difference (2, -1, 0, ...)
    g = gk_recurrence(2.0, 10)
    assert np.allclose(g, [2.0, -1.0] + [0.0] * 8, atol=1e-15)
    assert np.allclose(gk_closed_form(2.0, 10), g, atol=1e-15)


@pytest.mark.parametrize("gam", (1.2, 1.5, 1.8))
def test_fourier_coefficients_of_symbol(gam):
    # g_k are the Fourier coefficients of |2 sin(theta/2)|^gam (the generating function of
    # the fractional centred difference): check with a fine FFT of the sampled symbol.
    n = 2**20
    theta = 2 * np.pi * np.arange(n) / n
    coef = np.fft.fft(np.abs(2 * np.sin(theta / 2)) ** gam).real / n
    g = gk_recurrence(gam, 16)
    assert np.max(np.abs(coef[:16] - g)) < 1e-7
