"""The allocation-free adjoint entry point (vct_apply_ops_adjoint_noalloc),
called through the C ABI, against vct_apply_ops_adjoint with a caller
workspace (push form, the same kernels): bit-identical dphi and dtheta on two
calls in a row, the second on a smaller particle set, so that the second call
runs on the scratch the first one left behind."""
import ctypes as C

import numpy as np
import pytest

from paper_2607_28872_amd import inputs as I
from paper_2607_28872_amd import vct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
MASK = vct.VCT_OUT_LAP | vct.VCT_OUT_PZ


def _p(t):
    return C.c_void_p(t.data_ptr())


def _both(w):
    g = vct.Geometry(w.pos, w.vol, w.lo, w.hi, w.R, w.kernel, device=DEV, keep_col=False)
    g.moments(w.mapspec, MASK)
    proj = g.apply(g.sorted_field(w.phi[0]), vct.VCT_FP64)
    u = 2.0 * (proj[0, : g.n, 0] - g.sorted_field(np.cos(3.0 * w.pos[0]))[0])
    dphi_ws, dth_ws = g.adjoint(u, proj)
    nt = g.cmap.nterms
    dphi = torch.full((g.n,), float("nan"), dtype=torch.float64, device=DEV)
    dth = torch.full((max(nt, 1),), float("nan"), dtype=torch.float64, device=DEV)
    st = vct.lib().vct_apply_ops_adjoint_noalloc(C.byref(g.nl), _p(g.pos), _p(g.vol), g.kernel, _p(g.state64), MASK,
                                                 C.byref(g.cmap), _p(proj), _p(u), _p(dphi), _p(dth),
                                                 C.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == vct.VCT_OK, vct.status_string(st)
    return dphi_ws, dth_ws, dphi, dth[:nt]


def test_noalloc_adjoint_equals_the_workspace_entry_point_on_two_calls():
    first = I.small("sigma3d")          # 10,080 particles
    second = I.small("sigma3d-adj")     # 4,400 particles, 16 more bathymetry terms
    assert second.n < first.n
    for w in (first, second):
        d_ws, t_ws, d_na, t_na = _both(w)
        print(f"\n{w.name}: n={w.n}, max|dphi| {float(d_ws.abs().max()):.3e}")
        assert torch.equal(d_ws, d_na)
        assert torch.equal(t_ws, t_na)
        assert torch.isfinite(d_na).all()


def test_noalloc_adjoint_rejects_a_set_beyond_its_scratch():
    w = I.small("sigma3d")
    g = vct.Geometry(w.pos, w.vol, w.lo, w.hi, w.R, w.kernel, device=DEV, keep_col=False)
    nl = vct.vct_nlist.from_buffer_copy(g.nl)
    nl.n = 1 << 24   # 16.8M particles: the push form's workspace exceeds 64 MiB
    st = vct.lib().vct_apply_ops_adjoint_noalloc(C.byref(nl), None, None, 0, None, MASK, C.byref(vct.make_map(w.mapspec)),
                                                 None, None, None, None, None)
    assert st == vct.VCT_E_CAPACITY
