"""Build libvct.so (HIP, gfx950) in-tree.

Each translation unit under csrc/ is compiled with hipcc for gfx950 only, then
linked into paper_2607_28872_amd/libvct.so.  Packed FP32 instructions are
disabled (-packed-fp32-ops), and with them the straight-line vectoriser, whose
two-wide FP32 groups would only be split again and cost registers; FP64 contraction is left to the compiler except
where the source turns it off (the neighbour test).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvct.so")
BUILD_DIR = os.path.join(ROOT, "_build")
SOURCES = ["api.hip", "cells.hip", "moments.hip", "apply.hip", "adjoint.hip", "ppe.hip", "isph.hip", "jbar.hip"]
ROCM = "/opt/rocm"
HIPCC = os.environ.get("HIPCC", os.path.join(ROCM, "bin", "hipcc"))
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-fno-slp-vectorize",
          "-I", os.path.join(ROOT, "include")]


# Host-side sanitizers for the library's host code (argument checks, map
# set-up, workspace carving, launch timing); device code is not instrumented.
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
            "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


CHECKED_LIB = os.path.join(HERE, "libvct_checked.so")


def build(verbose: bool = False, extra=None, sanitize_host: bool = False, out=None, checks: bool = False) -> str:
    """Compile and link the library.  sanitize_host=True builds the host code
    with AddressSanitizer and UndefinedBehaviorSanitizer into `out` (default
    _build/libvct_san.so), for runs with the clang ASan runtime preloaded
    (VCT_LIB names it to the binding).  checks=True builds the debug library
    with device bounds checks (VCT_DEVICE_CHECKS=1) into `out` (default
    libvct_checked.so beside libvct.so; VCT_LIB names it to the binding)."""
    sub = "san" if sanitize_host else "checked" if checks else None
    build_dir = os.path.join(BUILD_DIR, sub) if sub else BUILD_DIR
    os.makedirs(build_dir, exist_ok=True)
    extra = list(extra or []) + (HOST_SAN if sanitize_host else []) + (["-DVCT_DEVICE_CHECKS=1"] if checks else [])
    lib_out = out or (os.path.join(build_dir, "libvct_san.so") if sanitize_host else CHECKED_LIB if checks else LIB)

    def compile_one(src):
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = lib_out + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", *(HOST_SAN if sanitize_host else []), *objs, "-o", tmp,
           "-L", os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib_out)
    return lib_out


if __name__ == "__main__":
    print(build(verbose=True))
