"""Fractional centred-difference weights omega_l^(gamma) (Section 2.1, eq. (2.4)).

Named g_k in the library: g_k = omega_k^(gamma), and g_{-k} = g_k (Lemma 2.1).
"""
from __future__ import annotations

import numpy as np
from scipy.special import gamma as _gamma, gammaln, gammasgn


def gk_recurrence(gam: float, n: int) -> np.ndarray:
    """g_0..g_{n-1} from eq. (2.4) via the ratio of consecutive weights.

    eq. (2.4): omega_l = (-1)^l Gamma(1+gam) / (Gamma(1+gam/2-l) Gamma(1+gam/2+l)).
    With Gamma(z+1) = z Gamma(z) the ratio omega_{l+1}/omega_l equals
    (l - gam/2) / (l + 1 + gam/2), and omega_0 = Gamma(1+gam) / Gamma(1+gam/2)^2.
    """
    g = np.empty(n, dtype=np.float64)
    if n == 0:
        return g
    g[0] = _gamma(1.0 + gam) / _gamma(1.0 + gam / 2.0) ** 2
    for k in range(n - 1):
        g[k + 1] = g[k] * (k - gam / 2.0) / (k + 1.0 + gam / 2.0)
    return g


def gk_closed_form(gam: float, n: int) -> np.ndarray:
    """g_0..g_{n-1} evaluated directly from eq. (2.4) with log-Gamma and its sign.

    Gamma(1+gam/2-l) has negative arguments for large l, so the value is formed as
    (-1)^l * sign * exp(lnGamma(1+gam) - ln|Gamma(1+gam/2-l)| - lnGamma(1+gam/2+l)).
    At a pole of Gamma(1+gam/2-l) (gam = 2, l >= 2) the weight is 0.
    """
    l = np.arange(n, dtype=np.float64)
    z = 1.0 + gam / 2.0 - l
    sgn = gammasgn(z)
    with np.errstate(over="ignore", invalid="ignore"):
        mag = np.exp(gammaln(1.0 + gam) - gammaln(z) - gammaln(1.0 + gam / 2.0 + l))
    out = np.where(np.isfinite(gammaln(z)), ((-1.0) ** l) * sgn * mag, 0.0)
    # at poles gammaln = +inf and exp(-inf) = 0 already; guard nan from sgn = 0
    return np.nan_to_num(out, nan=0.0)


def gk_tail_sum_asymptote(gam: float, K: int) -> float:
    """Leading-order value of g_0 + 2 sum_{k=1}^{K} g_k for large K.

    Lemma 2.1 gives sum over all integers = 0, so the partial sum equals
    -2 sum_{k>K} g_k.  The reflection formula turns eq. (2.4) into
    g_k = -Gamma(1+gam) sin(pi gam / 2) Gamma(k - gam/2) / (pi Gamma(k + 1 + gam/2))
    ~ -Gamma(1+gam) sin(pi gam/2) / pi * k^(-1-gam), whose tail sum is
    Gamma(1+gam) sin(pi gam/2) / (pi gam) * K^(-gam).
    """
    return 2.0 * _gamma(1.0 + gam) * np.sin(np.pi * gam / 2.0) / (np.pi * gam) * K ** (-gam)
