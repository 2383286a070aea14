"""Helpers shared by the GPU tests (host-side marshalling only)."""
import numpy as np

TOL_FFT = 1e-12     # FFT-based products: rounding ~ u log2(L) relative to the operand norm
TOL_SOLVE = 1e-10   # shifted solves / preconditioner: rounding times cond(B_n) at these sizes


def torch_mod():
    import torch
    return torch


def to_dev(x: np.ndarray, dtype=None):
    torch = torch_mod()
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def rel_max(a: np.ndarray, b: np.ndarray) -> float:
    """max |a - b| / max |b| (elementwise comparison, normalised by the reference's size)."""
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def banner(msg: str):
    print(f"[case] {msg}", flush=True)
