"""Seeded synthetic inputs and the workload shapes of the benchmarked configurations.

This module is shared by the tests, the benchmark and the GPU smoke check.  It holds
no arithmetic of the solution method: it only draws seeded random coefficients and
samples smooth sine-mode fields on the interior grid points, so that the oracle and
the HIP path receive bit-identical inputs.

Grid convention (Section 2.1): the interval (a, b) is split into M + 1 cells,
h = (b - a) / (M + 1), interior nodes x_i = a + i h for i = 1..M; the time grid is
t_k = k tau, tau = T / N_t, and the unknowns are u^1..u^{N_t} (t_1..t_{N_t}).

Data recipe (the paper's examples are closed-form manufactured solutions, not a
dataset; these fields stand in for "smooth initial data and source"):
  gen1d(seed): a_k, b_k = N(0,1) / k^2 for k = 1..8 from numpy default_rng(seed),
               a first, then b;  u0(x_i) = sum_k a_k sin(k pi (x_i - a)/(b - a));
               f(x_i, t_j) = exp(-t_j) sum_k b_k sin(k pi (x_i - a)/(b - a)), j = 1..N_t.
  gen2d(seed): a_kl, b_kl = N(0,1) / (k^2 l^2), k, l = 1..8, with the products
               sin(k pi x) sin(l pi y); layout [y][x] with x fastest.
"""
from __future__ import annotations

import numpy as np
from scipy.special import gamma as G

N_MODES = 8


def grid_1d(a: float, b: float, M: int) -> np.ndarray:
    """Interior nodes x_1..x_M of (a, b) with h = (b - a)/(M + 1)."""
    h = (b - a) / (M + 1)
    return a + h * np.arange(1, M + 1, dtype=np.float64)


def time_levels(T: float, Nt: int) -> np.ndarray:
    """t_1..t_{N_t} with tau = T / N_t."""
    tau = T / Nt
    return tau * np.arange(1, Nt + 1, dtype=np.float64)


def gen1d(seed: int, M: int, Nt: int, T: float = 1.0, a: float = 0.0, b: float = 1.0):
    """Seeded 1D initial data u0[M] and source f[N_t][M] (float64)."""
    rng = np.random.default_rng(seed)
    k = np.arange(1, N_MODES + 1, dtype=np.float64)
    ak = rng.standard_normal(N_MODES) / k**2
    bk = rng.standard_normal(N_MODES) / k**2
    x = grid_1d(a, b, M)
    modes = np.sin(np.pi * np.outer(k, (x - a) / (b - a)))  # [8][M]
    u0 = ak @ modes
    t = time_levels(T, Nt)
    f = np.exp(-t)[:, None] * (bk @ modes)[None, :]
    return np.ascontiguousarray(u0), np.ascontiguousarray(f), (ak, bk)


def gen2d(seed: int, Mx: int, My: int, Nt: int, T: float = 1.0,
          ax: float = 0.0, bx: float = 1.0, ay: float = 0.0, by: float = 1.0):
    """Seeded 2D initial data u0[My][Mx] and source f[N_t][My][Mx] (float64, x fastest)."""
    rng = np.random.default_rng(seed)
    k = np.arange(1, N_MODES + 1, dtype=np.float64)
    w = 1.0 / np.outer(k**2, k**2)  # [k(x)][l(y)]
    akl = rng.standard_normal((N_MODES, N_MODES)) * w
    bkl = rng.standard_normal((N_MODES, N_MODES)) * w
    x = grid_1d(ax, bx, Mx)
    y = grid_1d(ay, by, My)
    sx = np.sin(np.pi * np.outer(k, (x - ax) / (bx - ax)))  # [k][Mx]
    sy = np.sin(np.pi * np.outer(k, (y - ay) / (by - ay)))  # [l][My]
    u0 = sy.T @ akl.T @ sx          # [My][Mx] = sum_kl a_kl sy[l,y] sx[k,x]
    g = sy.T @ bkl.T @ sx
    t = time_levels(T, Nt)
    f = np.exp(-t)[:, None, None] * g[None, :, :]
    return np.ascontiguousarray(u0), np.ascontiguousarray(f), (akl, bkl)


def random_vector(seed: int, n: int) -> np.ndarray:
    """Seeded N(0,1) test vector (used to probe linear operators)."""
    return np.random.default_rng(seed).standard_normal(n)


# Workload shapes.  Each entry is the problem statement (eq. (1.1) / eq. (4.1)) plus
# solver settings; 'seed' feeds gen1d / gen2d.
SMALL_1D = dict(name="1d_M63_Nt64", dim=1, alpha=1.5, kappa=1.0, a=0.0, b=1.0,
                M=63, Nt=64, T=1.0, tol=1e-10, seed=1000)
LARGE_1D = dict(name="1d_M4095_Nt1024", dim=1, alphas=(1.2, 1.5, 1.8), kappa=1.0,
                a=0.0, b=1.0, M=4095, Nt=1024, T=1.0, tol=1e-8, seed=2000)
GRID_2D = dict(name="2d_255x255_Nt256", dim=2, alpha_x=1.6, alpha_y=1.4,
               kappa_x=1.0, kappa_y=1.0, Mx=255, My=255, Nt=256, T=1.0,
               tol=1e-8, seed=3000)


def batched_1d_instances(n: int = 64, seed: int = 4):
    """Uneven 1D instances: M ~ U{511..4095}, N_t ~ U{128..1024},
    alpha ~ U(1.1, 1.9), kappa ~ LogNormal(0, 0.5), drawn in that order."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        M = int(rng.integers(511, 4096))
        Nt = int(rng.integers(128, 1025))
        alpha = float(rng.uniform(1.1, 1.9))
        kappa = float(rng.lognormal(0.0, 0.5))
        out.append(dict(M=M, Nt=Nt, alpha=alpha, kappa=kappa, T=1.0, seed=4000 + i))
    return out


# ---------------------------------------------------------------------------------------------
# The paper's two test problems (Section 4): closed-form manufactured solutions and the source
# terms that produce them.  They define problem data (inputs), not solver arithmetic.


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


# ---------------------------------------------------------------------------------------------
# Learned initial guess: parameter draws and unit data components (inputs only).

LEARNED = dict(name="1d_M1023_Nt512_learned", M=1023, Nt=512, T=1.0, Ks=64, nsrc=16,
               train_points=625, train_seed=5000, heldout_seed=15000)


def learned_param_draw(seed: int):
    """alpha ~ U(1.1, 1.9), kappa ~ LogNormal(0, 0.5) from numpy default_rng(seed), in that order."""
    rng = np.random.default_rng(seed)
    return float(rng.uniform(1.1, 1.9)), float(rng.lognormal(0.0, 0.5))


def learned_instance(seed: int, M: int, Nt: int, T: float = 1.0):
    """A held-out instance: (alpha, kappa) as learned_param_draw, then gen1d data with the same
    seed.  Returns alpha, kappa, u0, f, coefficient vector c = (a_1..a_8, b_1..b_8)."""
    alpha, kappa = learned_param_draw(seed)
    u0, f, (ak, bk) = gen1d(seed, M, Nt, T)
    return alpha, kappa, u0, f, np.concatenate([ak, bk])


def unit_data(k: int, M: int, Nt: int, T: float = 1.0):
    """Unit data component k = 0..15: k < 8 -> u0 = sin((k+1) pi x), f = 0; k >= 8 ->
    u0 = 0, f = exp(-t) sin((k-7) pi x).  The gen1d data are sum_k c_k unit_data(k)."""
    x = grid_1d(0.0, 1.0, M)
    t = time_levels(T, Nt)
    mode = (k % N_MODES) + 1
    s = np.sin(mode * np.pi * x)
    if k < N_MODES:
        return s.copy(), np.zeros((Nt, M))
    return np.zeros(M), np.exp(-t)[:, None] * s[None, :]
