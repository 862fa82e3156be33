"""GPU parity of the volume smoothing of the sigma method (Sec. 3.6,
Eq. VCT_bar_a) against the oracle's sequential update, through the C ABI.

vct_jbar_smooth visits the target particles cell by cell in 3^d phases
(documented with the entry point); the oracle runs the paper's sequential
update with the targets in that same order and each row's neighbours in
ascending sorted index.  The order is built here from the definition of the
background-cell grid (cell coordinates, the sort by cell key and original
index), not from anything the library returns.  The two evaluate the same
exchanges in different roundings (closed-form Jbar updates against J / Jbar
values and a prefix scan); every exchange is a convex combination, so the
differences stay at the level of a few ulps per exchange: bar 1e-12 of each
particle's Jbar.  Also checked: conservation of sum J / Jbar on the GPU, a
set whose cell blocks exceed the LDS area (updated in memory), the full
2.1M-particle sigma set, and C_V = 0.
"""
import numpy as np
import pytest

import oracle as O
from paper_2607_28872_amd import inputs as I
from paper_2607_28872_amd import vct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
BAR = 1e-12
CV = 1e-2


def _cells(pos, lo, hi, R):
    """Cell coordinates (dim, n) and cell keys of the background grid."""
    dim, n = pos.shape
    _, dims = vct.vct_grid_dims(dim, lo, hi, R)
    coords = []
    for a in range(dim):
        ext = hi[a] - lo[a]
        nc = dims[a]
        inv = float(nc) / ext
        t = np.floor((pos[a] - lo[a]) * inv)
        t = np.where(t >= 0.0, t, 0.0)
        t = np.minimum(t, nc - 1)
        coords.append(t.astype(np.int64))
    if dim == 3:
        key = (coords[0] * dims[1] + coords[1]) * dims[2] + coords[2]
        colour = coords[0] % 3 + 3 * (coords[1] % 3) + 9 * (coords[2] % 3)
    else:
        key = coords[0] * dims[1] + coords[1]
        colour = coords[0] % 3 + 3 * (coords[1] % 3)
    return key, colour


def _oracle_in_schedule_order(w, J, jb0, cv):
    """The oracle's sequential update with the targets in the library's
    phase order.  The particles are relabelled in sorted order (cell key,
    then original index), so the oracle's rows, ascending in the new labels,
    are in ascending sorted index; the targets are then the sorted order
    stably reordered by phase."""
    key, colour = _cells(w.pos, w.lo, w.hi, w.R)
    srt = np.lexsort((np.arange(w.n), key))
    pos = np.ascontiguousarray(w.pos[:, srt])
    csr = O.neighbors(pos, w.R)
    order = np.argsort(colour[srt], kind="stable")
    ref = np.empty(w.n)
    ref[srt] = O.jbar_smooth(pos, J[srt], jb0[srt], cv, w.R, order=order, csr=csr)
    return ref


def _run(w, J, jb0, cv):
    g = vct.Geometry(w.pos, w.vol, w.lo, w.hi, w.R, w.kernel, device=DEV, keep_col=False)
    Js = g.sorted_field(J)[0].contiguous()
    jbs = g.sorted_field(jb0)[0].contiguous()
    g.jbar_smooth(Js, jbs, cv)
    got = g.unsort(jbs[: g.n]).cpu().numpy()
    return got, _oracle_in_schedule_order(w, J, jb0, cv)


def _check(label, w, J, jb0, got, ref):
    err = np.abs(got - ref) / np.abs(ref)
    moved = np.abs(ref - jb0).max() / np.abs(jb0).max()
    v0, v1 = np.sum(J / jb0), np.sum(J / got)
    print(f"\n{label}: n={w.n} max relative error {err.max():.2e} (bar {BAR:.0e}), largest change {moved:.1e}, "
          f"volume drift {abs(v1 - v0) / v0:.1e}")
    assert err.max() <= BAR
    assert abs(v1 - v0) <= 1e-12 * v0
    assert moved > 1e-4


def _sigma_J(w):
    return O.alpha_beta(3, w.pos[0], w.pos[1], w.mapspec)[:, 0]


@pytest.mark.parametrize("family", ["bf2d", "bfe2d", "sigma3d"])
def test_jbar_matches_the_sequential_update(family):
    w = I.small(family)
    if w.dim == 3:
        J = _sigma_J(w)
    else:   # the 2-D maps have a constant alpha; any positive determinant will do
        J = 1.0 + 0.3 * np.random.default_rng(3).uniform(size=w.n)
    jb0 = J * I.volume_perturbation(w.n)
    got, ref = _run(w, J, jb0, CV)
    _check(w.name, w, J, jb0, got, ref)


def test_jbar_blocks_beyond_the_lds_area():
    """R = 5 dx: about 27 x 125 particles around each cell, more than the
    2,048 values staged in LDS, so the blocks are updated in memory."""
    w = I.make_sigma3d(24, 22, 14, 0.05, name="jbar-dense", nx_span=24)
    w.R = 5.0 * w.dx
    J = _sigma_J(w)
    jb0 = J * I.volume_perturbation(w.n)
    got, ref = _run(w, J, jb0, CV)
    _check("jbar-dense (R = 5 dx)", w, J, jb0, got, ref)


def test_jbar_full_sigma_set():
    """The 2.1M-particle sigma set, every particle."""
    w = I.config("c2")
    J = _sigma_J(w)
    jb0 = J * I.volume_perturbation(w.n)
    got, ref = _run(w, J, jb0, CV)
    _check("c2", w, J, jb0, got, ref)


def test_jbar_without_smoothing_is_the_identity():
    w = I.small("sigma3d")
    J = _sigma_J(w)
    jb0 = J * I.volume_perturbation(w.n)
    g = vct.Geometry(w.pos, w.vol, w.lo, w.hi, w.R, w.kernel, device=DEV, keep_col=False)
    jbs = g.sorted_field(jb0)[0].contiguous()
    g.jbar_smooth(g.sorted_field(J)[0].contiguous(), jbs, 0.0)
    got = g.unsort(jbs[: g.n]).cpu().numpy()
    assert np.abs(got - jb0).max() <= 4.5e-16 * np.abs(jb0).max()


@pytest.mark.parametrize("family", ["bf2d", "bfe2d", "sigma3d"])
def test_map_alpha_matches_oracle(family):
    """vct_map_alpha (J = det J = alpha, Eq. det_jacobi) against the oracle's
    mapping at every particle."""
    w = I.small(family)
    pos = torch.as_tensor(w.pos, device=DEV).contiguous()
    out = torch.empty(w.n, dtype=torch.float64, device=DEV)
    vct.vct_map_alpha(w.dim, w.n, pos, vct.make_map(w.mapspec), out)
    ref = O.alpha_beta(w.dim, w.pos[0], w.pos[1] if w.dim == 3 else None, w.mapspec)[:, 0]
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-14 * np.abs(ref).max()
