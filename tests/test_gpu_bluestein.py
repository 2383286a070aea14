"""GPU parity for time-level counts N_t that are not powers of two (steps (a) and (c) through
Bluestein's chirp-z form), against the FP64 oracle, whose time DFTs are numpy's for any length.
Odd N_t has no self-conjugate Nyquist level; even N_t has one."""
import numpy as np
import pytest

from gpu_util import TOL_FFT, TOL_SOLVE, banner, rel_max, to_dev, to_host
from oracle import allatonce as aa
from oracle import precond as pc
from oracle import twod
from rfde_workloads import gen1d, gen2d, random_vector

pytestmark = pytest.mark.gpu

STEP_CASES = [  # (alpha, M, Nt): transform lengths 8 .. 8192
    (1.5, 37, 3),
    (1.3, 63, 5),
    (1.7, 100, 6),
    (1.5, 64, 12),
    (1.8, 129, 100),
    (1.2, 65, 127),
    (1.5, 511, 1000),
    (1.6, 15, 4095),
]


def _plan(alpha, M, Nt, **kw):
    from paper_2003_07020_amd.rfde import Plan
    return Plan.create_1d(alpha, 1.0, 0.0, 1.0, M, Nt, 1.0, **kw)


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("alpha,M,Nt", STEP_CASES)
def test_time_steps_any_length(alpha, M, Nt, bits):
    banner(f"bluestein steps bits={bits} alpha={alpha} M={M} Nt={Nt}")
    p = _plan(alpha, M, Nt, precond_bits=bits)
    assert p.info["n_freq"] == Nt // 2 + 1
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    eps = pc.default_eps(tau)
    v = random_vector(71, Nt * M).reshape(Nt, M)
    z1 = to_host(p.step_a(to_dev(v.ravel()))).reshape(-1, M).astype(np.complex128)
    z1_ref = pc.step_a(v, eps)
    # FP32: rounding ~ u32 log2(Lt) over three transforms of length Lt <= 8192
    tol = TOL_FFT if bits == 64 else 2e-5
    assert rel_max(z1, z1_ref) < tol
    # the ABI takes complex128 half spectra and narrows them itself for an FP32 plan; step (c)
    # divides level j by s_j >= eps, which magnifies the transform's rounding (unit roundoff u)
    # by up to 1/eps
    vc = to_host(p.step_c(to_dev(z1_ref.ravel()))).reshape(Nt, M)
    u = 2.0**-53 if bits == 64 else 2.0**-24
    tol_c = max(tol, 16 * u / eps)
    assert rel_max(vc, pc.step_c(z1_ref, Nt, eps)) < tol_c
    if bits == 64:
        A = aa.jacobian_A(alpha, 1.0, h, M)
        z = to_host(p.apply_Pinv(to_dev(v.ravel()))).reshape(Nt, M)
        assert rel_max(z, pc.pinv_fast(v, A, tau, eps)) < TOL_SOLVE
        if Nt * M <= 2500:
            assert rel_max(z, pc.pinv_dense(v, A, tau, eps)) < TOL_SOLVE


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("alpha,M,Nt", [(1.5, 63, 100), (1.8, 100, 127), (1.3, 300, 257)])
def test_solve_any_length(alpha, M, Nt, bits):
    banner(f"bluestein solve bits={bits} alpha={alpha} M={M} Nt={Nt}")
    p = _plan(alpha, M, Nt, precond_bits=bits, tol=1e-11)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    u0, f, _ = gen1d(72, M, Nt)
    U, st, _ = p.solve(to_dev(u0), to_dev(f.ravel()))
    U = to_host(U).reshape(Nt, M)
    assert st.converged and st.true_rel_res <= 1e-11
    assert rel_max(U, aa.bdf2_march(u0, f, aa.jacobian_A(alpha, 1.0, h, M), tau)) < 1e-9


@pytest.mark.parametrize("bits", [64, 32])
def test_solve_2d_any_length(bits):
    gx, gy, Mx, My, Nt = 1.6, 1.4, 15, 31, 100
    banner(f"bluestein 2d solve bits={bits} {Mx}x{My} Nt={Nt}")
    from paper_2003_07020_amd.rfde import Plan
    p = Plan.create_2d(gx, gy, 1.0, 1.0, 0.0, 1.0, 0.0, 1.0, Mx, My, Nt, 1.0, precond_bits=bits)
    hx, hy, tau = 1.0 / (Mx + 1), 1.0 / (My + 1), 1.0 / Nt
    Tx, Ty = aa.toeplitz_T(gx, Mx), aa.toeplitz_T(gy, My)
    cx, cy = twod.coeffs(gx, gy, 1.0, 1.0, hx, hy)
    u0, f, _ = gen2d(73, Mx, My, Nt)
    U, st, _ = p.solve(to_dev(u0.ravel()), to_dev(f.ravel()), tol=1e-11)
    U = to_host(U).reshape(Nt, My, Mx)
    assert st.converged and st.true_rel_res <= 1e-11
    assert rel_max(U, twod.bdf2_march_2d(u0, f, Tx, Ty, cx, cy, tau)) < 1e-9
