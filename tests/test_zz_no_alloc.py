"""The entry point that allocates nothing (rfde_mlp_forward_noalloc) against the workspace entry
point it varies (rfde_mlp_forward): same kernels, so the outputs must agree bit for bit, on two
calls in a row (the second with a smaller batch and a smaller network, which reuses the fixed
device array the first call left behind), plus its argument checks."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu


def _make(seed, Pin, H1, H2, NOUT):
    from paper_2003_07020_amd.learned import GuessNet
    rng = np.random.default_rng(seed)
    mu = rng.standard_normal(Pin) * 0.1
    sd = 1.0 + rng.random(Pin)
    net = GuessNet(Pin, H1, H2, NOUT, mu, sd, seed=seed, init_scale=1.0, max_batch=64)
    return net, rng


@pytest.mark.parametrize("first,second", [
    ((64, 19, 256, 256, 4096), (5, 3, 64, 128, 1024)),   # largest activations, then smaller
    ((32, 3, 128, 256, 2048), (1, 3, 128, 256, 2048)),   # same network, smaller batch
])
def test_noalloc_forward_matches_workspace_forward(first, second):
    import torch
    for call, (B, Pin, H1, H2, NOUT) in enumerate((first, second)):
        banner(f"mlp forward noalloc call {call}: B={B} Pin={Pin} H1={H1} H2={H2} NOUT={NOUT}")
        net, rng = _make(100 + call, Pin, H1, H2, NOUT)
        feats = to_dev(rng.standard_normal((B, Pin)).astype(np.float32))
        ref = to_host(net.forward(feats)).copy()
        out = torch.full((B * NOUT,), float("nan"), dtype=torch.float32, device="cuda")
        got = to_host(net.forward_noalloc(feats, out))
        torch.cuda.synchronize()
        assert np.all(np.isfinite(got))
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), call


def test_noalloc_forward_rejects_invalid_arguments():
    from paper_2003_07020_amd import capi
    from paper_2003_07020_amd.learned import _bind
    from paper_2003_07020_amd.rfde import _ptr, _stream
    import torch
    lib = _bind()
    assert lib.rfde_mlp_forward_noalloc_max_bytes() == 256 * 1024
    net, rng = _make(7, 3, 16, 32, 64)
    feats = to_dev(rng.standard_normal((65, 3)).astype(np.float32))
    out = torch.empty(65 * 64, dtype=torch.float32, device="cuda")
    net._refresh_struct()
    # batch above 64, batch 0, missing output
    assert lib.rfde_mlp_forward_noalloc(C.byref(net.s), _ptr(feats), 65, _ptr(out),
                                        _stream()) == capi.RFDE_EINVAL
    assert lib.rfde_mlp_forward_noalloc(C.byref(net.s), _ptr(feats), 0, _ptr(out),
                                        _stream()) == capi.RFDE_EINVAL
    assert lib.rfde_mlp_forward_noalloc(C.byref(net.s), _ptr(feats), 4, None,
                                        _stream()) == capi.RFDE_EINVAL
    assert lib.rfde_mlp_forward_noalloc(None, _ptr(feats), 4, _ptr(out),
                                        _stream()) == capi.RFDE_EINVAL
