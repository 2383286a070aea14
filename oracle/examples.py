"""Manufactured solutions of Section 4 (Examples 1 and 2), used only to pin the oracle
against the error values printed in Tables 1-6."""
from __future__ import annotations

import numpy as np
from scipy.special import gamma as G


def example1_exact(gam, x, t):
    """u(x, t) = 15 (1 + gam/4) e^t x^3 (1 - x)^3 on (0, 1) (Example 1)."""
    return 15.0 * (1.0 + gam / 4.0) * np.exp(t) * x**3 * (1.0 - x) ** 3


def example1_source(gam, kappa, x, t):
    """Source term of Example 1, as printed (kappa = 0.01 in the paper)."""
    c = 15.0 * (1.0 + gam / 4.0)
    bracket = (G(4) / G(4 - gam) * (x ** (3 - gam) + (1 - x) ** (3 - gam))
               - 3 * G(5) / G(5 - gam) * (x ** (4 - gam) + (1 - x) ** (4 - gam))
               + 3 * G(6) / G(6 - gam) * (x ** (5 - gam) + (1 - x) ** (5 - gam))
               - G(7) / G(7 - gam) * (x ** (6 - gam) + (1 - x) ** (6 - gam)))
    return (c * np.exp(t) * x**3 * (1 - x) ** 3
            + c * kappa * np.exp(t) / (2.0 * np.cos(gam * np.pi / 2.0)) * bracket)


Q_EX2 = {5: 16.0, 6: -32.0, 7: 24.0, 8: -8.0, 9: 1.0}  # x^4 (2-x)^4 = sum q_l x^{l-1}


def example2_exact(x, y, t):
    """u(x, y, t) = e^{-t/3} x^4 (2-x)^4 y^4 (2-y)^4 on (0, 2)^2 (Example 2)."""
    return np.exp(-t / 3.0) * x**4 * (2 - x) ** 4 * y**4 * (2 - y) ** 4


def _riesz_poly_part(g, z):
    return sum(q * G(l) * (z ** (l - 1 - g) + (2 - z) ** (l - 1 - g)) / G(l - g)
               for l, q in Q_EX2.items())


def example2_source(g1, g2, k1, k2, x, y, t):
    """Source term of Example 2.  Reading: the third term's bracket is evaluated in y
    (the printed formula repeats x there; only the y reading matches the tabulated
    errors), and the exact solution is u(x, y, t)."""
    X = x**4 * (2 - x) ** 4
    Y = y**4 * (2 - y) ** 4
    e = np.exp(-t / 3.0)
    return (-e / 3.0 * X * Y
            + k1 * e / (2.0 * np.cos(g1 * np.pi / 2.0)) * Y * _riesz_poly_part(g1, x)
            + k2 * e / (2.0 * np.cos(g2 * np.pi / 2.0)) * X * _riesz_poly_part(g2, y))
