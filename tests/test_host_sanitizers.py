"""The host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer on the CPU:
a sanitizer build (host pass only) is loaded, with the sanitizer runtime preloaded, by the C-ABI
tests (argument validation before any device work, struct layouts, exported symbols); any
invalid access or undefined behaviour in those paths aborts the run."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_abi_checks_pass_under_host_sanitizers(tmp_path):
    from paper_2003_07020_amd import build as b
    try:
        b._hipcc()
        runtime = b.asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    lib = b.build(sanitize=True, out_dir=str(tmp_path), jobs=8)
    env = dict(os.environ)
    env.update(LD_PRELOAD=runtime, RFDE_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                          os.path.join(ROOT, "tests", "test_abi.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "passed" in res.stdout and "ERROR: AddressSanitizer" not in out
    assert "runtime error:" not in out  # UBSan reports
    shutil.rmtree(tmp_path / "obj", ignore_errors=True)
