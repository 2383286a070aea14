"""Build the HIP library librfde.so for gfx950 in-tree (hipcc, one object per source).

Usage: python -m paper_2003_07020_amd.build  (or call build()).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "librfde.so")
ARCH = os.environ.get("RFDE_OFFLOAD_ARCH", "gfx950")

# Packed FP32 instructions (v_pk_*_f32) are disabled for all device code; every kernel is
# validated with plain scalar FP32/FP64 arithmetic only.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the rfde library needs the ROCm toolchain")


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer for the CPU checks of the host code
# (argument validation, plan bookkeeping): every sanitizer flag applies to the host pass only;
# the device code is compiled as in the normal build.
HOST_SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, build_dir: str = BUILD, flags=None) -> str:
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [_hipcc(), *(HIP_FLAGS if flags is None else flags), "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    return obj


def build(verbose: bool = False, jobs: int = 8, sanitize: bool = False,
          out_dir: str | None = None) -> str:
    """Compile every csrc/*.hip for gfx950 and link librfde.so (always rebuilds).

    sanitize=True builds the host code under AddressSanitizer and UndefinedBehaviorSanitizer
    (-O1 -g) into out_dir/librfde_hostsan.so instead (out_dir required: keep it outside the
    tree); load it with the sanitizer runtime preloaded (`asan_runtime()`) and RFDE_LIBRARY
    naming it."""
    if sanitize:
        if not out_dir:
            raise ValueError("a sanitizer build needs out_dir")
        build_dir = os.path.join(out_dir, "obj")
        lib_path = os.path.join(out_dir, "librfde_hostsan.so")
        flags = [f for f in HIP_FLAGS if f != "-O3"] + ["-O1", "-g", *HOST_SAN_FLAGS]
        link_extra = [*HOST_SAN_FLAGS, "-shared-libsan"]
    else:
        build_dir, lib_path, flags, link_extra = BUILD, LIB, HIP_FLAGS, []
    os.makedirs(build_dir, exist_ok=True)
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, flags), srcs))
    tmp = lib_path + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *link_extra, *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, lib_path)
    if verbose:
        print(f"built {lib_path}")
    return lib_path


def asan_runtime() -> str:
    """Path of the compiler's shared AddressSanitizer runtime (to preload into the host
    process that loads a sanitizer build)."""
    res = subprocess.run([_hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = res.stdout.strip()
    if res.returncode != 0 or not os.path.isfile(path):
        raise RuntimeError("AddressSanitizer runtime not found")
    return path


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
