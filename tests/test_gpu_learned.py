"""GPU tests of the learned initial guess: forward / gradients / Adam of the hand-written network
kernels against the FP64 oracle, the sine projection and guess assembly, and an end-to-end
check that the trained guess lowers the FGMRES iteration count (zero-guess fallback included)."""
import numpy as np
import pytest

from gpu_util import banner, rel_max, to_dev, to_host
from oracle import allatonce as aa
from oracle import mlp as omlp
import rfde_workloads as wl

pytestmark = pytest.mark.gpu


def _bf16_round(a):
    """Round float32 values to the nearest BF16-representable value (test input generation)."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _small_net(seed, Pin=3, H1=8, H2=32, NOUT=96):
    from paper_2003_07020_amd.learned import GuessNet
    rng = np.random.default_rng(seed)
    host = [rng.standard_normal((H1, Pin)).astype(np.float32) * 0.6,
            rng.standard_normal(H1).astype(np.float32) * 0.1,
            rng.standard_normal((H2, H1)).astype(np.float32) * 0.4,
            rng.standard_normal(H2).astype(np.float32) * 0.1,
            _bf16_round(rng.standard_normal((NOUT, H2)) * 0.3),
            rng.standard_normal(NOUT).astype(np.float32) * 0.1]
    mu = np.array([0.1, -0.2, 0.3, 0.05][:Pin], np.float32)
    sd = np.array([1.5, 0.7, 2.0, 1.1][:Pin], np.float32)
    net = GuessNet(Pin, H1, H2, NOUT, mu, sd)
    net.set_params(host)
    p = rng.standard_normal((5, Pin)).astype(np.float32)
    y = rng.standard_normal((5, NOUT)).astype(np.float32)
    params64 = [h.astype(np.float64) for h in host]
    return net, params64, p, y, mu.astype(np.float64), sd.astype(np.float64)


def test_forward_and_gradients_match_oracle():
    banner("mlp forward/grads")
    net, P, p, y, mu, sd = _small_net(1)
    g = to_host(net.forward(to_dev(p)))
    g_ref = omlp.forward(P, p.astype(np.float64), mu, sd)[3]
    # BF16 copy of h2 in the output product: relative error ~ 2^-9
    assert rel_max(g, g_ref) < 1e-2
    grads, loss = net.grads(to_dev(p), to_dev(y))
    ref = omlp.grads(P, p.astype(np.float64), y.astype(np.float64), mu, sd)
    assert abs(float(loss.item()) / omlp.loss(P, p.astype(np.float64), y.astype(np.float64), mu, sd) - 1) < 1e-2
    for a, (gg, rr) in enumerate(zip(grads, ref)):
        gg = to_host(gg).astype(np.float64)
        err = np.linalg.norm(gg - rr) / np.linalg.norm(rr)
        assert err < 2e-2, (a, err)


def test_gradients_with_unaligned_output_match_oracle():
    """Pin = 2, H1 = 5: the output layer's block of the flat gradient starts at float 207, not on
    a 16-byte boundary, so its gradients are written one value per access."""
    banner("mlp grads, unaligned output layer block")
    net, P, p, y, mu, sd = _small_net(4, Pin=2, H1=5)
    grads, _ = net.grads(to_dev(p), to_dev(y))
    ref = omlp.grads(P, p.astype(np.float64), y.astype(np.float64), mu, sd)
    for a, (gg, rr) in enumerate(zip(grads, ref)):
        gg = to_host(gg).astype(np.float64)
        assert np.linalg.norm(gg - rr) / np.linalg.norm(rr) < 2e-2, a


def test_adam_step_unaligned_output_weights_bitwise():
    """The output layer's weights and Adam moments moved 4 bytes off a 16-byte boundary take the
    one-value-per-access path of the update; it must give the same bits as the aligned one."""
    import torch
    banner("mlp adam, unaligned output weights")
    made = [_small_net(5) for _ in range(2)]
    nets = [m[0] for m in made]
    p, y = made[0][2], made[0][3]
    net_u = nets[1]

    def shifted(t):
        buf = torch.zeros(t.numel() + 1, dtype=t.dtype, device=t.device)
        buf[1:].copy_(t.reshape(-1))
        return buf[1:].view(t.shape)

    net_u.params[4] = shifted(net_u.params[4])
    net_u.moments[8] = shifted(net_u.moments[8])
    net_u.moments[9] = shifted(net_u.moments[9])
    assert net_u.params[4].data_ptr() % 16 == 4
    for net in nets:
        for _ in range(3):
            net.train_step(to_dev(p), to_dev(y), 1e-3)
    for a, b in zip(nets[0].params, nets[1].params):
        assert np.array_equal(to_host(a), to_host(b))
    assert np.array_equal(to_host(nets[0].W3b), to_host(nets[1].W3b))


def test_adam_step_matches_oracle():
    banner("mlp adam")
    net, P, p, y, mu, sd = _small_net(2)
    lr = 1e-3
    net.train_step(to_dev(p), to_dev(y), lr)
    ref = omlp.grads(P, p.astype(np.float64), y.astype(np.float64), mu, sd)
    for a, (w, gr) in enumerate(zip(net.params, ref)):
        w1, _, _ = omlp.adam_step(P[a], gr, np.zeros_like(gr), np.zeros_like(gr), 1, lr)
        # the first Adam step moves each weight by ~lr * sign(grad); where the gradient is not
        # tiny the GPU and oracle steps agree, elsewhere the sign may differ within rounding
        d = np.abs(to_host(w).astype(np.float64) - w1)
        big = np.abs(gr) > 0.05 * np.abs(gr).max()
        assert np.all(d[big] < 0.05 * lr + 1e-6), a
        assert np.all(d <= 2.05 * lr + 1e-6), a


def test_projection_and_assembly():
    from paper_2003_07020_amd import learned as ln
    import torch
    banner("sine projection/assembly")
    lib = ln._bind()
    from paper_2003_07020_amd.rfde import _ptr, _stream
    M, Nt, Ks, nsrc = 63, 8, 16, 3
    S = torch.empty(M * Ks, dtype=torch.float64, device="cuda")
    assert lib.rfde_sine_table(M, Ks, _ptr(S), _stream()) == 0
    assert rel_max(to_host(S).reshape(M, Ks), omlp.sine_basis(M, Ks)) < 1e-14
    U = np.random.default_rng(3).standard_normal((Nt, M))
    Y = torch.empty(Nt * Ks, dtype=torch.float32, device="cuda")
    Ud = to_dev(U.ravel())
    assert lib.rfde_project_sine(Nt, M, Ks, _ptr(Ud), _ptr(S), 0.5, _ptr(Y), _stream()) == 0
    assert rel_max(to_host(Y).reshape(Nt, Ks), 0.5 * omlp.project(U, Ks)) < 1e-6
    g = np.random.default_rng(4).standard_normal(nsrc * Nt * Ks).astype(np.float32)
    coef = np.array([0.5, -1.0, 2.0])
    out = torch.empty(Nt * M, dtype=torch.float64, device="cuda")
    gd, cd = to_dev(g), to_dev(coef)
    assert lib.rfde_guess_assemble(nsrc, Nt, Ks, M, _ptr(gd), _ptr(cd), _ptr(S), _ptr(out),
                                   _stream()) == 0
    ref = omlp.guess(g.astype(np.float64), coef, np.ones(nsrc), Nt, Ks, M)
    assert rel_max(to_host(out).reshape(Nt, M), ref) < 1e-12


def test_learned_guess_reduces_iterations():
    from paper_2003_07020_amd.learned import LearnedGuess
    from paper_2003_07020_amd.rfde import Plan
    import torch
    M, Nt, Ks = 63, 64, 16
    banner(f"learned guess end to end M={M} Nt={Nt}")
    units = [wl.unit_data(j, M, Nt) for j in range(16)]
    lg = LearnedGuess(M, Nt, units, Ks=Ks, H1=32, H2=64, seed=0)
    draws = [wl.learned_param_draw(5000 + i) for i in range(48)]
    feats, Y, nsolve = lg.generate(draws)
    assert nsolve == 48 * 16
    hist = lg.train(feats, Y, epochs=300, batch=16, lr0=3e-3, lr1=3e-5)
    it0, it1, errs = [], [], []
    for s in range(15000, 15008):
        alpha, kappa, u0, f, c = wl.learned_instance(s, M, Nt)
        with Plan.create_1d(alpha, kappa, 0.0, 1.0, M, Nt, 1.0, tol=1e-10) as p:
            U0, st0, _ = p.solve(to_dev(u0), to_dev(f.ravel()))
            Ug = lg.guess(alpha, kappa, c)
            U1, st1, _ = p.solve(to_dev(u0), to_dev(f.ravel()), U_init=Ug)
            h, tau = aa.mesh(0, 1, M, 1.0, Nt)
            Uref = aa.bdf2_march(u0, f, aa.jacobian_A(alpha, kappa, h, M), tau)
            errs.append(np.linalg.norm(to_host(Ug) - Uref.ravel()) / np.linalg.norm(Uref))
            assert st1.converged and rel_max(to_host(U1).reshape(Nt, M), Uref) < 1e-8
            it0.append(st0.iters)
            it1.append(st1.iters)
    print(f"learned: guess rel err median {np.median(errs):.2e}, iters zero {np.mean(it0):.2f} "
          f"-> guess {np.mean(it1):.2f}", flush=True)
    assert np.median(errs) < 0.05
    assert np.mean(it1) < np.mean(it0)


def test_bad_guess_falls_back_to_zero():
    from paper_2003_07020_amd.rfde import Plan
    M, Nt = 63, 16
    banner("guess fallback")
    u0, f, _ = wl.gen1d(7, M, Nt)
    with Plan.create_1d(1.5, 1.0, 0.0, 1.0, M, Nt, 1.0, tol=1e-10) as p:
        _, st0, _ = p.solve(to_dev(u0), to_dev(f.ravel()))
        bad = to_dev(np.full(Nt * M, 1e6))
        U, st1, _ = p.solve(to_dev(u0), to_dev(f.ravel()), U_init=bad)
        assert st1.converged and st1.iters == st0.iters


def test_learned_guess_at_benchmark_shape():
    # the learned-guess workload's own shape (M = 1023, N_t = 512, Ks = 64 sine modes) with a
    # reduced training set (48 parameter draws = 768 method-generated FP64 solves): the guess
    # must land within 5% of the oracle's solution, and the guessed solves must take no more
    # iterations than the zero start and still reach the FP64 bar.  (At this training size the
    # guess is 2-5% off; its residual ||F - A U_g|| is then several times ||F||, because the
    # all-at-once matrix amplifies the error in the higher sine modes, so the solver falls back
    # to the zero start.  The benchmark trains on 625 draws and reports the iterations saved
    # over 1000 held-out instances.)
    from paper_2003_07020_amd.learned import LearnedGuess
    from paper_2003_07020_amd.rfde import Plan
    LW = wl.LEARNED
    M, Nt, Ks = LW["M"], LW["Nt"], LW["Ks"]
    banner(f"learned guess at M={M} Nt={Nt} Ks={Ks}")
    units = [wl.unit_data(j, M, Nt) for j in range(16)]
    lg = LearnedGuess(M, Nt, units, Ks=Ks, H1=64, H2=128, seed=0)
    draws = [wl.learned_param_draw(LW["train_seed"] + i) for i in range(48)]
    feats, Y, nsolve = lg.generate(draws)
    assert nsolve == 48 * 16
    lg.train(feats, Y, epochs=400, batch=16, lr0=2e-3, lr1=2e-5)
    del Y
    it0, it1, errs, res0 = [], [], [], []
    for s in range(LW["heldout_seed"], LW["heldout_seed"] + 4):
        alpha, kappa, u0, f, c = wl.learned_instance(s, M, Nt)
        h, tau = aa.mesh(0, 1, M, 1.0, Nt)
        Uref = aa.bdf2_march(u0, f, aa.jacobian_A(alpha, kappa, h, M), tau)
        with Plan.create_1d(alpha, kappa, 0.0, 1.0, M, Nt, 1.0, tol=1e-8) as p:
            _, st0, _ = p.solve(to_dev(u0), to_dev(f.ravel()))
            Ug = lg.guess(alpha, kappa, c)
            U1, st1, _ = p.solve(to_dev(u0), to_dev(f.ravel()), U_init=Ug)
            # relative residual of the guess itself, ||F - A U_g|| / ||F||
            F = p.build_rhs(to_dev(u0), to_dev(f.ravel()))
            r0 = float((F - p.apply_A(Ug)).norm() / F.norm())
        assert np.isfinite(r0)
        res0.append(r0)
        errs.append(np.linalg.norm(to_host(Ug) - Uref.ravel()) / np.linalg.norm(Uref))
        assert st1.converged and st1.true_rel_res <= 1e-8
        assert rel_max(to_host(U1).reshape(Nt, M), Uref) < 1e-8
        it0.append(st0.iters)
        it1.append(st1.iters)
    print(f"learned at M={M}: guess rel err median {np.median(errs):.2e}, guess residual "
          f"median {np.median(res0):.2e}, iters zero {np.mean(it0):.2f} -> guess "
          f"{np.mean(it1):.2f}", flush=True)
    assert np.median(errs) < 0.05
    assert np.mean(it1) <= np.mean(it0)
