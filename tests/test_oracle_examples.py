"""Pins of the oracle against the numbers printed in Tables 1-6 (Section 4) and the
second-order temporal convergence of the BDF2 scheme (Section 2.1)."""
import csv
import os

import numpy as np
import pytest

from oracle import allatonce as aa
from oracle import krylov
from oracle import precond as pc
from oracle import twod
from oracle.weights import gk_recurrence
import rfde_workloads as ex

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return list(csv.DictReader(line for line in fh if not line.startswith("#")))


def _example1(gam, Nt, N, kappa=0.01):
    M, h, tau = N - 1, 1.0 / N, 1.0 / Nt
    x = h * np.arange(1, M + 1)
    t = tau * np.arange(1, Nt + 1)
    A = aa.jacobian_A(gam, kappa, h, M)
    u0 = ex.example1_exact(gam, x, 0.0)
    f = ex.example1_source(gam, kappa, x[None, :], t[:, None])
    return x, A, u0, f, tau, M


def _gmres_tau(A_, u0, f, tau, gam, kappa, h, M, Nt, eps):
    sig = -(kappa / h**gam) * pc.tau_eigenvalues(gk_recurrence(gam, M))
    F = aa.rhs_F(u0, f, tau).ravel()
    Av = lambda v: aa.apply_all_at_once(v.reshape(Nt, M), A_, tau).ravel()
    Mv = lambda v: pc.pinv_tau(v.reshape(Nt, M), sig, tau, eps).ravel()
    x, info = krylov.fgmres(Av, Mv, F, tol=1e-9)
    it = next(i for i, r in enumerate(info["history"]) if r < 1e-9)
    return x.reshape(Nt, M), it, np.log10(info["true_rel_res"])


@pytest.mark.parametrize("row", _rows("example1_tables.csv"),
                         ids=lambda r: f"T{r['table']}-g{r['gamma']}-Nt{r['Nt']}-N{r['N']}")
def test_tables_1_to_3(row):
    gam, Nt, N = float(row["gamma"]), int(row["Nt"]), int(row["N"])
    x, A, u0, f, tau, M = _example1(gam, Nt, N)
    h = 1.0 / N
    # P_alpha: iteration count exactly, log10 TRR to the printed 3 decimals, Err to 4 digits
    U, it, trr = _gmres_tau(A, u0, f, tau, gam, 0.01, h, M, Nt, pc.default_eps(tau))
    assert it == int(row["pa_iter"])
    assert abs(trr - float(row["pa_trr"])) <= 1.5e-3
    err = np.max(np.abs(U[-1] - ex.example1_exact(gam, x, 1.0)))
    assert abs(err / float(row["pa_err"]) - 1) < 5e-4
    # Err of the exact all-at-once solution (sequential BDF2) agrees to the same digits
    Ustar = aa.bdf2_march(u0, f, A, tau)
    errs = np.max(np.abs(Ustar[-1] - ex.example1_exact(gam, x, 1.0)))
    assert abs(errs / float(row["pa_err"]) - 1) < 5e-4
    # P_1: counts exact for gamma 1.2 and 1.9; at gamma 1.5 the printed P_1 counts are
    # reproduced to within one iteration (the P_1 runs are rounding-sensitive: lambda_0 = 0)
    _, it1, _ = _gmres_tau(A, u0, f, tau, gam, 0.01, h, M, Nt, 1.0)
    if gam in (1.2, 1.9):
        assert it1 == int(row["p1_iter"])
    else:
        assert abs(it1 - int(row["p1_iter"])) <= 1


@pytest.mark.parametrize("row", _rows("example2_tables.csv"),
                         ids=lambda r: f"T{r['table']}-Nt{r['Nt']}-N{r['N']}")
def test_tables_4_to_6_error(row):
    g1, g2, Nt, N = float(row["gamma1"]), float(row["gamma2"]), int(row["Nt"]), int(row["N"])
    Lx, T, k = 2.0, 2.0, 0.01
    M, h, tau = N - 1, Lx / N, T / Nt
    x = h * np.arange(1, M + 1)
    t = tau * np.arange(1, Nt + 1)
    Tx, Ty = aa.toeplitz_T(g1, M), aa.toeplitz_T(g2, M)
    cx, cy = twod.coeffs(g1, g2, k, k, h, h)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = ex.example2_exact(X, Y, 0.0)
    f = ex.example2_source(g1, g2, k, k, X[None], Y[None], t[:, None, None])
    U = twod.bdf2_march_2d(u0, f, Tx, Ty, cx, cy, tau)
    err = np.max(np.abs(U[-1] - ex.example2_exact(X, Y, T)))
    assert abs(err / float(row["pa_err"]) - 1) < 5e-4


@pytest.mark.parametrize("gam", (1.2, 1.8))
def test_second_order_in_time(gam):
    # Section 2.1: BDF2 with a backward-Euler start is second order in tau; at a fine
    # spatial grid the Example 1 error drops by ~4 per halving of tau
    N = 1024
    errs = []
    for Nt in (8, 16, 32):
        x, A, u0, f, tau, M = _example1(gam, Nt, N, kappa=0.01)
        U = aa.bdf2_march_eig(u0, f, A, tau)
        errs.append(np.max(np.abs(U[-1] - ex.example1_exact(gam, x, 1.0))))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5
