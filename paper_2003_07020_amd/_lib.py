"""ctypes binding of include/rfde.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librfde.so")

RFDE_OK = 0
RFDE_ENOTCONV = 1
RFDE_EINVAL = -1
RFDE_ENOMEM = -2
RFDE_EHIP = -3
RFDE_ENAN = -4
RFDE_EUNSUPPORTED = -5

SPATIAL_EXACT = 0
SPATIAL_TAU = 1
SPATIAL_TOEPLITZ = 2

(EXPORT_GK, EXPORT_SYMBOL, EXPORT_LAMBDA, EXPORT_SCALE, EXPORT_FACTOR, EXPORT_TAU_SIGMA,
 EXPORT_TOEPLITZ_X) = range(7)


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int), ("restart", C.c_int),
                ("circ_eps", C.c_double), ("precond_bits", C.c_int), ("spatial", C.c_int),
                ("inner_iters", C.c_int), ("inner_tol", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("converged", C.c_int),
                ("true_rel_res", C.c_double), ("ms_setup", C.c_double), ("ms_solve", C.c_double),
                ("n_pinv", C.c_int), ("n_matvec", C.c_int), ("ms_pinv_est", C.c_double),
                ("ms_matvec_est", C.c_double), ("n_hist", C.c_int),
                ("res_hist", C.c_double * 256)]


class PlanInfo(C.Structure):
    _fields_ = [("dim", C.c_int), ("M", C.c_int), ("Mx", C.c_int), ("My", C.c_int),
                ("Nt", C.c_int), ("n_freq", C.c_int), ("L", C.c_int), ("Lx", C.c_int),
                ("Ly", C.c_int), ("Mp", C.c_int), ("h", C.c_double), ("hx", C.c_double),
                ("hy", C.c_double), ("tau", C.c_double), ("circ_eps", C.c_double),
                ("coef", C.c_double), ("coef_x", C.c_double), ("coef_y", C.c_double),
                ("factor_bytes", C.c_size_t), ("workspace_bytes", C.c_size_t),
                ("precond_bits", C.c_int), ("spatial", C.c_int), ("ms_setup", C.c_double),
                ("ms_factor", C.c_double)]


class Instance(C.Structure):
    _fields_ = [("alpha", C.c_double), ("kappa", C.c_double), ("a", C.c_double),
                ("b", C.c_double), ("T", C.c_double), ("M", C.c_int), ("Nt", C.c_int)]


class BatchInfo(C.Structure):
    _fields_ = [("count", C.c_int), ("waves", C.c_int), ("max_wave", C.c_int),
                ("budget_bytes", C.c_size_t), ("wave_bytes_max", C.c_size_t),
                ("instance_bytes_max", C.c_size_t),
                ("device_bytes_max", C.c_size_t), ("ms_setup", C.c_double),
                ("ms_plans", C.c_double), ("ms_tune", C.c_double),
                ("ms_factor", C.c_double), ("ms_solve", C.c_double),
                ("graph_launches", C.c_int)]


class TuneReport(C.Structure):
    _fields_ = [("time_variant", C.c_int), ("matvec_variant", C.c_int),
                ("trsv_grid_cap", C.c_int), ("from_cache", C.c_int),
                ("ms_time", C.c_double * 4), ("ms_matvec", C.c_double * 4),
                ("trsv_caps", C.c_int * 5), ("ms_trsv", C.c_double * 5)]


class RfdeError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} (status {code})")


_lib = None


def lib() -> C.CDLL:
    """Load librfde.so (built in-tree); raise if it is missing -- there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    # RFDE_LIBRARY names another build of the same library (e.g. one compiled with different
    # launch shapes); the default is the in-tree build
    path = os.environ.get("RFDE_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2003_07020_amd.build` (needs hipcc, gfx950)")
    L = C.CDLL(path)
    vp, dp, ip, d, i = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_double, C.c_int
    L.rfde_opts_default.argtypes = [C.POINTER(Opts)]
    L.rfde_opts_default.restype = None
    L.rfde_strerror.argtypes = [i]
    L.rfde_strerror.restype = C.c_char_p
    L.rfde_gk.argtypes = [d, i, vp, vp]
    L.rfde_plan_create_1d.argtypes = [C.POINTER(vp), d, d, d, d, i, i, d, C.POINTER(Opts), vp]
    L.rfde_plan_create_2d.argtypes = [C.POINTER(vp), d, d, d, d, d, d, d, d, i, i, i, d,
                                      C.POINTER(Opts), vp]
    L.rfde_plan_destroy.argtypes = [vp]
    L.rfde_plan_get_info.argtypes = [vp, C.POINTER(PlanInfo)]
    L.rfde_plan_export.argtypes = [vp, i, i, vp]
    L.rfde_build_rhs.argtypes = [vp, vp, vp, vp]
    L.rfde_apply_A.argtypes = [vp, vp, vp]
    L.rfde_pinv_step_a.argtypes = [vp, vp, vp]
    L.rfde_pinv_step_b.argtypes = [vp, vp, vp]
    L.rfde_pinv_step_c.argtypes = [vp, vp, vp]
    L.rfde_apply_Pinv.argtypes = [vp, vp, vp]
    L.rfde_solve.argtypes = [vp, vp, vp, vp, vp, d, C.POINTER(Stats)]
    L.rfde_plan_autotune.argtypes = [vp, C.POINTER(TuneReport)]
    L.rfde_release_cached_memory.argtypes = []
    L.rfde_release_cached_memory.restype = C.c_size_t
    L.rfde_plan_set_variants.argtypes = [vp, i, i, i]
    L.rfde_batch_create.argtypes = [C.POINTER(vp), i, C.POINTER(Instance), C.POINTER(Opts),
                                    C.c_size_t, vp]
    L.rfde_batch_solve.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                   C.POINTER(Stats)]
    L.rfde_batch_set_grid_caps.argtypes = [vp, i, i]
    L.rfde_batch_set_autotune.argtypes = [vp, i]
    L.rfde_batch_wave_of.argtypes = [vp, i]
    L.rfde_batch_get_info.argtypes = [vp, C.POINTER(BatchInfo)]
    L.rfde_batch_destroy.argtypes = [vp]
    L.rfde_probe_mfma.argtypes = [i, i, C.POINTER(d), vp]
    for name in ("rfde_probe_mfma", "rfde_gk", "rfde_plan_create_1d", "rfde_plan_create_2d", "rfde_plan_destroy",
                 "rfde_plan_get_info", "rfde_plan_export", "rfde_build_rhs", "rfde_apply_A",
                 "rfde_pinv_step_a", "rfde_pinv_step_b", "rfde_pinv_step_c", "rfde_apply_Pinv",
                 "rfde_solve", "rfde_plan_autotune", "rfde_plan_set_variants", "rfde_batch_create", "rfde_batch_solve", "rfde_batch_set_grid_caps", "rfde_batch_set_autotune",
                 "rfde_batch_wave_of", "rfde_batch_get_info", "rfde_batch_destroy"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().rfde_strerror(int(code)).decode()
    except RuntimeError:
        return f"status {code}"


def check(code: int, where: str, allow=(RFDE_OK,)) -> int:
    if code not in allow:
        raise RfdeError(code, where)
    return code
