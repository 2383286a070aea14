"""The C-ABI library loads, exports every function declared in include/rfde.h, and rejects
invalid arguments before touching the device (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rfde.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rfde_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("rfde_gk", "rfde_plan_create_1d", "rfde_plan_create_2d", "rfde_build_rhs",
              "rfde_apply_A", "rfde_pinv_step_a", "rfde_pinv_step_b", "rfde_pinv_step_c",
              "rfde_apply_Pinv", "rfde_solve", "rfde_plan_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2003_07020_amd import lib
    L = lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_invalid_arguments_rejected_without_device():
    from paper_2003_07020_amd import capi
    L = capi.lib()
    h = C.c_void_p()
    bad = [
        (0.9, 1.0, 0.0, 1.0, 63, 64, 1.0),    # alpha <= 1
        (2.1, 1.0, 0.0, 1.0, 63, 64, 1.0),    # alpha > 2
        (1.5, 0.0, 0.0, 1.0, 63, 64, 1.0),    # kappa <= 0
        (1.5, 1.0, 1.0, 1.0, 63, 64, 1.0),    # b <= a
        (1.5, 1.0, 0.0, 1.0, 0, 64, 1.0),     # M < 1
        (1.5, 1.0, 0.0, 1.0, 5000, 64, 1.0),  # M too large
        (1.5, 1.0, 0.0, 1.0, 63, 1, 1.0),     # Nt < 2
        (1.5, 1.0, 0.0, 1.0, 63, 4097, 1.0),  # Nt not a power of two and above 4096
        (1.5, 1.0, 0.0, 1.0, 63, 16384, 1.0), # Nt above 8192
        (1.5, 1.0, 0.0, 1.0, 63, 64, 0.0),    # T <= 0
    ]
    for args in bad:
        rc = L.rfde_plan_create_1d(C.byref(h), *args, None, None)
        assert rc == capi.RFDE_EINVAL, args
        assert h.value is None
    o = capi.Opts()
    L.rfde_opts_default(C.byref(o))
    assert o.tol == 1e-8 and o.restart == 30 and o.precond_bits == 64
    for field, val in (("circ_eps", 1.5), ("precond_bits", 16), ("restart", 0), ("tol", -1.0)):
        o2 = capi.Opts()
        L.rfde_opts_default(C.byref(o2))
        setattr(o2, field, val)
        rc = L.rfde_plan_create_1d(C.byref(h), 1.5, 1.0, 0.0, 1.0, 63, 64, 1.0, C.byref(o2), None)
        assert rc == capi.RFDE_EINVAL, field
    assert L.rfde_gk(1.5, 0, None, None) == capi.RFDE_EINVAL
    assert L.rfde_gk(2.5, 5, C.c_void_p(8), None) == capi.RFDE_EINVAL
    assert L.rfde_apply_A(None, None, None) == capi.RFDE_EINVAL
    assert L.rfde_solve(None, None, None, None, None, 0.0, None) == capi.RFDE_EINVAL
    assert L.rfde_plan_destroy(None) == capi.RFDE_OK
    # 2D grid sizes above 4096 per axis
    rc = L.rfde_plan_create_2d(C.byref(h), 1.6, 1.4, 1.0, 1.0, 0.0, 1.0, 0.0, 1.0, 5000, 255, 256,
                               1.0, None, None)
    assert rc == capi.RFDE_EINVAL
    assert L.rfde_strerror(capi.RFDE_ENAN).decode().startswith("non-finite")


def test_inner_solver_options_validated_without_device():
    # the optional inner solver of the 2D step (b): 0..16 steps, tolerance >= 0, 2D and the
    # FP64 preconditioner only
    from paper_2003_07020_amd import capi
    L = capi.lib()
    h = C.c_void_p()

    def opts(**kw):
        o = capi.Opts()
        L.rfde_opts_default(C.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return o
    assert opts().inner_iters == 0 and opts().inner_tol == 0.0
    for kw in ({"inner_iters": -1}, {"inner_iters": 17}, {"inner_iters": 2, "inner_tol": -1.0},
               {"inner_iters": 2, "inner_tol": float("nan")}):
        o = opts(**kw)
        rc = L.rfde_plan_create_2d(C.byref(h), 1.6, 1.4, 1.0, 1.0, 0.0, 1.0, 0.0, 1.0, 15, 7, 8,
                                   1.0, C.byref(o), None)
        assert rc == capi.RFDE_EINVAL, kw
        assert h.value is None
    o = opts(inner_iters=2, precond_bits=32)
    assert L.rfde_plan_create_2d(C.byref(h), 1.6, 1.4, 1.0, 1.0, 0.0, 1.0, 0.0, 1.0, 15, 7, 8, 1.0,
                                 C.byref(o), None) == capi.RFDE_EUNSUPPORTED
    o = opts(inner_iters=2, spatial=1)
    assert L.rfde_plan_create_1d(C.byref(h), 1.5, 1.0, 0.0, 1.0, 63, 16, 1.0, C.byref(o),
                                 None) == capi.RFDE_EUNSUPPORTED
    arr = (capi.Instance * 1)(capi.Instance(1.5, 1.0, 0.0, 1.0, 1.0, 63, 64))
    o = opts(inner_iters=2)
    assert L.rfde_batch_create(C.byref(h), 1, arr, C.byref(o), 0, None) == capi.RFDE_EUNSUPPORTED
    assert h.value is None


def test_batch_rejects_invalid_arguments_without_device():
    from paper_2003_07020_amd import capi
    L = capi.lib()
    h = C.c_void_p()
    good = capi.Instance(1.5, 1.0, 0.0, 1.0, 1.0, 63, 64)
    bad = capi.Instance(1.5, 1.0, 0.0, 1.0, 1.0, 63, 4097)
    arr = (capi.Instance * 2)(good, bad)
    assert L.rfde_batch_create(C.byref(h), 0, arr, None, 0, None) == capi.RFDE_EINVAL
    assert L.rfde_batch_create(C.byref(h), 2, None, None, 0, None) == capi.RFDE_EINVAL
    assert L.rfde_batch_create(C.byref(h), 2, arr, None, 0, None) == capi.RFDE_EINVAL
    assert h.value is None
    o = capi.Opts()
    L.rfde_opts_default(C.byref(o))
    o.spatial = 1
    assert L.rfde_batch_create(C.byref(h), 1, arr, C.byref(o), 0, None) == capi.RFDE_EUNSUPPORTED
    assert L.rfde_batch_solve(None, None, None, None, None) == capi.RFDE_EINVAL
    assert L.rfde_batch_destroy(None) == capi.RFDE_OK


def _c_layout(struct, fields):
    """sizeof and offsetof of a header struct, from a C program compiled with the host gcc."""
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    body = "".join(f'  printf("%zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src = (f'#include <stdio.h>\n#include <stddef.h>\n#include "rfde.h"\nint main(void) {{\n'
           f'  printf("%zu\\n", sizeof({struct}));\n{body}  return 0;\n}}\n')
    with tempfile.TemporaryDirectory() as d:
        c, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(c, "w").write(src)
        subprocess.run([cc, "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


@pytest.mark.parametrize("struct,pyname", [("rfde_opts", "Opts"), ("rfde_stats", "Stats"),
                                           ("rfde_plan_info", "PlanInfo"),
                                           ("rfde_instance", "Instance"),
                                           ("rfde_batch_info", "BatchInfo")])
def test_binding_structs_match_header_layout(struct, pyname):
    # every field of the header's struct, in order, at the same offset, same total size
    from paper_2003_07020_amd import capi
    py = getattr(capi, pyname)
    names = [f for f, _ in py._fields_]
    size, offs = _c_layout(struct, names)
    assert C.sizeof(py) == size
    assert [getattr(py, f).offset for f in names] == offs
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct\s*\{([^}]*)\}\s*" + struct + r"\s*;", src).group(1)
    declared = re.findall(r"([A-Za-z_][A-Za-z0-9_]*)\s*(?:\[[^\]]*\])?\s*[;,]", body)
    assert declared == names
