"""GPU parity of the 1D variants: the FP32 preconditioner (complex64 LDL^T on FP32 MFMA inside
FP64 FGMRES) and the tau/DST step (b) (the paper's own implementation), including the
iteration counts of Tables 1-3 reproduced by the GPU solver."""
import csv
import os

import numpy as np
import pytest

import paper_2003_07020_amd._lib as capi

from gpu_util import banner, rel_max, to_dev, to_host
from oracle import allatonce as aa
from oracle import precond as pc
from oracle.weights import gk_recurrence
import rfde_workloads as wl

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _plan(alpha, kappa, M, Nt, **kw):
    from paper_2003_07020_amd.rfde import Plan
    return Plan.create_1d(alpha, kappa, 0.0, 1.0, M, Nt, 1.0, **kw)


@pytest.mark.parametrize("alpha,M,Nt", [(1.5, 63, 64), (1.8, 200, 16), (1.2, 130, 32)])
def test_fp32_factor_and_solve(alpha, M, Nt):
    from paper_2003_07020_amd import capi
    banner(f"fp32 alpha={alpha} M={M} Nt={Nt}")
    p = _plan(alpha, 1.0, M, Nt, precond_bits=32, tol=1e-11)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    A = aa.jacobian_A(alpha, 1.0, h, M)
    eps = pc.default_eps(tau)
    lam = pc.eigenvalues(Nt, eps)
    Mp = p.info["Mp"]
    for n in (0, Nt // 2):
        F = to_host(p.export(capi.EXPORT_FACTOR, n)).reshape(Mp, Mp).astype(np.complex128)
        Lf = np.tril(F, -1) + np.eye(Mp)
        B = Lf @ np.diag(np.diag(F)) @ Lf.T
        ref = np.eye(Mp, dtype=complex)
        ref[:M, :M] = pc.shifted_matrix(lam[n], A, tau)
        assert rel_max(B, ref) < 1e-5
    v = wl.random_vector(41, Nt * M).reshape(Nt, M)
    z1 = pc.step_a(v, eps)
    z2 = to_host(p.step_b(to_dev(z1.ravel()))).reshape(-1, M)
    ref = pc.step_b_exact(z1, A, tau, Nt, eps)
    # FP32 error ~ u32 * cond(B_n) (cond <= 1e4 here)
    assert rel_max(z2, ref) < 1e-3
    u0, f, _ = wl.gen1d(42, M, Nt)
    U, st, _ = p.solve(to_dev(u0), to_dev(f.ravel()))
    U = to_host(U).reshape(Nt, M)
    assert st.converged and st.true_rel_res <= 1e-11
    assert rel_max(U, aa.bdf2_march(u0, f, A, tau)) < 1e-9


@pytest.mark.parametrize("alpha,M,Nt", [(1.5, 63, 64), (1.2, 127, 8), (1.9, 255, 32),
                                         (1.6, 1023, 8), (1.4, 2047, 4), (1.8, 4095, 8),
                                         (1.7, 511, 7), (1.3, 1023, 5)])
@pytest.mark.parametrize("bits", [64, 32])
def test_tau_step_b_1d(alpha, M, Nt, bits):
    banner(f"tau1d bits={bits} alpha={alpha} M={M} Nt={Nt}")
    p = _plan(alpha, 1.0, M, Nt, spatial="tau", precond_bits=bits)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    eps = pc.default_eps(tau)
    g = gk_recurrence(alpha, M)
    # sigma_i = (Q chat)_i / Q_{i1} (eq. (3.10)) cancels heavily for the smallest eigenvalues at
    # large M (sigma_1 = 2.5e-6 from terms of size ~1e-2 at alpha = 1.8, M = 4095), so two FP64
    # evaluations in different summation orders agree only to the rounding bound of that sum:
    # |d sigma_i| <= (M + 4 log2 P) u sum_k |Q_ik chat_k| / |Q_i1| (dense sum in the oracle,
    # FFT of length P = 2(M+1) on the GPU).
    sig_gpu = to_host(p.export(capi.EXPORT_TAU_SIGMA))
    sig_or = pc.tau_eigenvalues(g)
    Q = pc.dst_matrix(M)
    bound = (np.abs(Q) @ np.abs(pc.tau_first_column(g))) / np.abs(Q[:, 0])
    u = np.finfo(np.float64).eps / 2
    assert np.all(np.abs(sig_gpu - sig_or) <= (M + 4 * np.log2(2 * (M + 1))) * u * bound)
    # step (b) itself, given the plan's sigma
    sig_A = -(1.0 / h**alpha) * sig_gpu
    v = wl.random_vector(43, Nt * M).reshape(Nt, M)
    z1 = pc.step_a(v, eps)
    z2 = to_host(p.step_b(to_dev(z1.ravel()))).reshape(-1, M)
    assert rel_max(z2, pc.step_b_tau(z1, sig_A, tau, Nt, eps)) < (1e-11 if bits == 64 else 2e-5)


def _rows():
    with open(os.path.join(GOLDEN, "example1_tables.csv")) as fh:
        rows = list(csv.DictReader(line for line in fh if not line.startswith("#")))
    return [r for r in rows if int(r["Nt"]) * int(r["N"]) <= 2**16]


@pytest.mark.parametrize("row", _rows(), ids=lambda r: f"g{r['gamma']}-Nt{r['Nt']}-N{r['N']}")
def test_tables_1_to_3_iterations_on_gpu(row):
    # Example 1 with the tau step (b): the GPU FGMRES stops after the printed P_alpha count
    gam, Nt, N = float(row["gamma"]), int(row["Nt"]), int(row["N"])
    M, h, tau = N - 1, 1.0 / N, 1.0 / Nt
    banner(f"table row gamma={gam} Nt={Nt} N={N}")
    x = h * np.arange(1, M + 1)
    t = tau * np.arange(1, Nt + 1)
    u0 = wl.example1_exact(gam, x, 0.0)
    f = wl.example1_source(gam, 0.01, x[None, :], t[:, None])
    p = _plan(gam, 0.01, M, Nt, spatial="tau", tol=1e-9)
    U, st, _ = p.solve(to_dev(u0), to_dev(f.ravel()), allow_notconv=True)
    hist = st.res_hist
    k = next(i for i, r in enumerate(hist) if r < 1e-9)
    assert k == int(row["pa_iter"])
    U = to_host(U).reshape(Nt, M)
    err = np.max(np.abs(U[-1] - wl.example1_exact(gam, x, 1.0)))
    assert abs(err / float(row["pa_err"]) - 1) < 5e-4
