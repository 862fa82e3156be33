"""The debug library with device bounds checks (libvct_checked.so, built with
VCT_DEVICE_CHECKS=1), run in child processes (tests/_checks_driver.py):

  * on a valid small sigma set every kernel family -- neighbour search,
    moments, FP64 and mixed applies, conventional operators, the field and
    bathymetry adjoints (both readings), the volume smoothing -- gives the
    same bits as the release library and sets no check;
  * a window offset set one past the end of its chunk's window is caught by
    the FP64 apply: the window bit is set and the kernel runs to its end (the
    index is replaced by one inside the window).  The planted offset is the
    first value past the window, whose record, were it read, still lies
    inside the buffers.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2607_28872_amd import build, vct

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "_checks_driver.py")


def _run(lib, mode, tmp_path):
    out = str(tmp_path / f"{os.path.basename(lib)}_{mode}.npz")
    env = dict(os.environ, VCT_LIB=lib)
    r = subprocess.run([sys.executable, "-u", DRIVER, out, mode], env=env, capture_output=True, text=True,
                       timeout=240)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0
    return dict(np.load(out))


@pytest.fixture(scope="module")
def libs():
    for p in (vct.LIB_PATH, build.CHECKED_LIB):
        if not os.path.exists(p):
            pytest.fail(f"{p} is not built (run __graft_entry__.build())")
    return vct.LIB_PATH, build.CHECKED_LIB


def test_checked_build_matches_release_bits_and_sets_no_check(libs, tmp_path):
    rel = _run(libs[0], "valid", tmp_path)
    chk = _run(libs[1], "valid", tmp_path)
    assert int(rel["checked"]) == 0 and int(rel["bits"]) == 0
    assert int(chk["checked"]) == 1
    assert int(chk["bits"]) == 0, f"device checks set: {int(chk['bits']):#x}"
    for k in rel:
        if k in ("checked", "bits"):
            continue
        assert np.array_equal(rel[k], chk[k], equal_nan=True), k


def test_checked_build_flags_an_offset_past_its_window(libs, tmp_path):
    res = _run(libs[1], "plant", tmp_path)
    i, e, W = (int(x) for x in res["planted"])
    print(f"\nplanted offset {W} (one past the window) at entry {e} of particle {i}")
    assert int(res["checked"]) == 1
    assert int(res["bits"]) & vct.VCT_CHECK_WINDOW
