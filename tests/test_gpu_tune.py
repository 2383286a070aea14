"""Launch-shape variants and the tuner: every variant of the time FFTs, the matvec and the
triangular solves computes the same result as the default shape (to rounding), and a tuned plan
still solves to the oracle's answer."""
import numpy as np
import pytest

from gpu_util import TOL_FFT, banner, rel_max, to_dev, to_host
from oracle import allatonce as aa
from oracle import precond as pc
from rfde_workloads import gen1d, random_vector

pytestmark = pytest.mark.gpu

SHAPES = [(1.5, 200, 64), (1.7, 129, 100), (1.3, 1000, 32)]


def _plan(alpha, M, Nt, **kw):
    from paper_2003_07020_amd.rfde import Plan
    return Plan.create_1d(alpha, 1.0, 0.0, 1.0, M, Nt, 1.0, **kw)


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("alpha,M,Nt", SHAPES)
def test_variants_agree(alpha, M, Nt, bits):
    banner(f"variants bits={bits} alpha={alpha} M={M} Nt={Nt}")
    p = _plan(alpha, M, Nt, precond_bits=bits)
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    A = aa.jacobian_A(alpha, 1.0, h, M)
    v = to_dev(random_vector(91, Nt * M))
    ref = {}
    for tv in range(4):
        for mv in range(4):
            for cap in (0, 7, 64):
                p.set_variants(tv, mv, cap)
                z1 = p.step_a(v)
                z2 = p.step_b(z1)
                vc = p.step_c(z2)
                y = p.apply_A(v)
                out = [to_host(t) for t in (z1, z2, vc, y)]
                if not ref:
                    ref = dict(z1=out[0], z2=out[1], vc=out[2], y=out[3])
                    y_or = aa.apply_all_at_once(to_host(v).reshape(Nt, M), A, tau)
                    assert rel_max(out[3].reshape(Nt, M), y_or) < TOL_FFT
                    continue
                # the same operations on each element; only the compiler's choice of fused
                # multiply-adds (and, for matvec variant 2, the radix) may differ between the
                # instantiations, so results agree to rounding
                tol = TOL_FFT if bits == 64 else 1e-5
                assert rel_max(out[0], ref["z1"]) < tol, (tv, mv, cap)
                assert rel_max(out[1], ref["z2"]) < tol, (tv, mv, cap)
                assert rel_max(out[2], ref["vc"]) < tol, (tv, mv, cap)
                assert rel_max(out[3], ref["y"]) < TOL_FFT, (tv, mv, cap)


@pytest.mark.parametrize("bits", [64, 32])
def test_autotuned_plan_solves(bits):
    banner(f"autotune bits={bits}")
    alpha, M, Nt = 1.6, 300, 100
    p = _plan(alpha, M, Nt, precond_bits=bits, tol=1e-11)
    rep = p.autotune()
    assert 0 <= rep["time_variant"] <= 3 and 0 <= rep["matvec_variant"] <= 3
    assert rep["trsv_grid_cap"] in rep["trsv_caps"]
    q = _plan(alpha, M, Nt, precond_bits=bits, tol=1e-11)
    rep2 = q.autotune()
    assert rep2["from_cache"] == 7
    assert (rep2["time_variant"], rep2["matvec_variant"], rep2["trsv_grid_cap"]) == \
        (rep["time_variant"], rep["matvec_variant"], rep["trsv_grid_cap"])
    h, tau = aa.mesh(0.0, 1.0, M, 1.0, Nt)
    u0, f, _ = gen1d(92, M, Nt)
    U, st, _ = p.solve(to_dev(u0), to_dev(f.ravel()))
    assert st.converged
    assert rel_max(to_host(U).reshape(Nt, M),
                   aa.bdf2_march(u0, f, aa.jacobian_A(alpha, 1.0, h, M), tau)) < 1e-9


def test_autotuned_batch_matches_untuned():
    from paper_2003_07020_amd.rfde import Batch
    banner("batch autotune")
    cases = [(1.5, 1.0, 100, 64), (1.25, 0.7, 77, 45), (1.85, 1.5, 160, 16)]
    inst = [dict(alpha=a, kappa=k, M=M, Nt=Nt) for a, k, M, Nt in cases]
    u0s, fs = [], []
    for i, (a, k, M, Nt) in enumerate(cases):
        u0, f, _ = gen1d(930 + i, M, Nt)
        u0s.append(to_dev(u0))
        fs.append(to_dev(f.ravel()))
    b0 = Batch(inst, tol=1e-10)
    U0, s0, _ = b0.solve(u0s, fs)
    b1 = Batch(inst, tol=1e-10)
    b1.set_autotune(3)
    U1, s1, _ = b1.solve(u0s, fs)
    for i, (a, k, M, Nt) in enumerate(cases):
        assert s1[i].converged
        assert rel_max(to_host(U1[i]), to_host(U0[i])) < 1e-9
