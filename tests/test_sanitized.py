"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

  * the oracle (orc.c) built with gcc -fsanitize=address,undefined runs every
    oracle pin (test_oracle.py, test_oracle_ppe.py, test_oracle_isph.py,
    test_oracle_jbar.py, test_oracle_r2.py, test_oracle_perparticle.py);
  * the library's host code (argument checks, map set-up, separable table,
    workspace carving, launch-timing registry) built with the same sanitizers
    on the host side only runs the ABI checks of test_abi.py.
Each run is a child process with the matching ASan runtime preloaded; any
report makes it exit non-zero.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(env_extra, *test_files):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"     # the interpreter itself is not instrumented
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *[os.path.join(ROOT, "tests", f) for f in test_files]], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, tail
    return r.stdout.strip().splitlines()[-1]


def _runtime(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True).stdout.strip()
    return p if p and os.path.exists(p) else None


def test_oracle_pins_under_asan_ubsan():
    import oracle
    rt = _runtime(["gcc", "-print-file-name=libasan.so"])
    if rt is None:
        pytest.skip("gcc ASan runtime not installed")
    lib = oracle.build(sanitize=True, out=os.path.join(ROOT, "_build", "liborc_san.so"))
    print(_run({"LD_PRELOAD": rt, "ORACLE_LIB": lib}, "test_oracle.py", "test_oracle_ppe.py", "test_oracle_isph.py",
         "test_oracle_jbar.py", "test_oracle_r2.py",
         "test_oracle_perparticle.py"))


def test_library_host_code_under_asan_ubsan():
    import glob
    from paper_2607_28872_amd import build as B
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rts:
        pytest.skip("clang ASan runtime not installed")
    lib = B.build(sanitize_host=True)
    print(_run({"LD_PRELOAD": rts[0], "VCT_LIB": lib}, "test_abi.py"))
