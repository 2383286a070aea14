"""MI355X (gfx950) all-at-once BDF2 solver for Riesz fractional diffusion equations with the
eps-circulant parallel-in-time preconditioner (arXiv:2003.07020).

The solver lives in the HIP library librfde.so (C ABI in include/rfde.h); this package is a
thin ctypes binding.  Importing it does not touch the GPU; using a plan requires the built
library and a gfx950 device, and fails loudly otherwise.
"""
from ._lib import RfdeError, lib  # noqa: F401
from . import _lib as capi  # noqa: F401

__all__ = ["RfdeError", "lib", "capi", "rfde"]


def __getattr__(name):
    if name == "rfde":
        from . import rfde as _r  # imports torch lazily
        return _r
    raise AttributeError(name)
