"""Pins of the oracle's bathymetry adjoint under reading R2 (physical
positions held fixed, so the projected heights z^ = alpha (z + beta) move with
the bathymetry coefficients; Sec. 2.1, Eq. VCT; Sec. 3.1, Eq. sec_SPH2).

The oracle differentiates the literal two-stage SPH(2) formula by the complex
step.  What pins it independently:
  * d loss / d z^_k against central differences of the real oracle's loss,
    z^_k moved by +-1e-6 R (the rows of k and its neighbours re-evaluated;
    the loss difference formed as (a - b)(a + b - 2 g) per row);
  * d loss / d coef_t against central differences of the real loss with the
    particles re-projected from their fixed physical positions;
  * the chain rule split: the total equals the fixed-projection sensitivity
    (reading R1, orc_dtheta) plus sum_k (d loss / d z^_k) (d z^_k / d coef_t);
  * translation invariance: with c_trans held, the SPH(2) derivatives do not
    change when every z^ moves by the same amount, so sum_k d loss / d z^_k
    vanishes.
"""
import numpy as np
import pytest

from paper_2607_28872_amd import inputs as I
import oracle as O


def _case(name):
    if name == "sigma3d":
        w = I.small("sigma3d-adj")
        tl = np.arange(len(w.mapspec.terms) - 16, len(w.mapspec.terms))
        g = w.extra["target"]
    else:
        w = I.small("bf2d")
        tl = np.arange(len(w.mapspec.terms))
        g = 100.0 * np.sin(2 * np.pi * w.pos[0])
    ab = O.alpha_beta(w.dim, w.pos[0], w.pos[1] if w.dim == 3 else None, w.mapspec)
    phys = w.pos.copy()
    phys[-1] = w.pos[-1] / ab[:, 0] - ab[:, 6]
    pos = O.project(phys, w.mapspec)       # the projected positions of those physical points
    csr = O.neighbors(pos, w.R)
    rec, fl = O.sph2(pos, w.vol, w.phi[0], w.kernel, w.R, w.mapspec, csr=csr)
    assert not fl.any()
    lap = rec[:, 0, O.I_LAP]
    return w, tl, g, phys, pos, csr, lap, 2.0 * (lap - g)


def _local_loss_diff(w, pos_p, pos_m, rows, csr, g):
    """sum over rows of (a - g)^2 - (b - g)^2 = (a - b)(a + b - 2 g)."""
    a = O.sph2(pos_p, w.vol, w.phi[0], w.kernel, w.R, w.mapspec, rows=rows, csr=_sub(csr, rows))[0][:, 0, O.I_LAP]
    b = O.sph2(pos_m, w.vol, w.phi[0], w.kernel, w.R, w.mapspec, rows=rows, csr=_sub(csr, rows))[0][:, 0, O.I_LAP]
    return float(np.sum((a - b) * (a + b - 2.0 * g[rows])))


def _sub(csr, rows):
    rp, col = csr
    deg = rp[rows + 1] - rp[rows]
    nrp = np.zeros(len(rows) + 1, dtype=np.int64)
    nrp[1:] = np.cumsum(deg)
    ncol = np.concatenate([col[rp[r]:rp[r + 1]] for r in rows]).astype(np.int32)
    return nrp, ncol


@pytest.mark.parametrize("name", ["sigma3d", "bf2d"])
def test_dzhat_matches_central_differences(orc, name):
    w, tl, g, phys, pos, csr, lap, u = _case(name)
    rng = np.random.default_rng(5)
    ks = rng.choice(w.n, 12, replace=False)
    got = O.r2_dzhat(pos, w.vol, w.phi[0], w.kernel, w.R, w.mapspec, u, ks=ks, csr=csr)
    h = 1e-6 * w.R
    rp, col = csr
    for k, gk in zip(ks, got):
        rows = np.concatenate([[k], col[rp[k]:rp[k + 1]]]).astype(np.int64)
        pp, pm = pos.copy(), pos.copy()
        pp[-1, k] += h
        pm[-1, k] -= h
        fd = _local_loss_diff(w, pp, pm, rows, csr, g) / (2 * h)
        assert abs(gk - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(got).max()), (k, gk, fd)


@pytest.mark.parametrize("name", ["sigma3d", "bf2d"])
def test_dtheta_matches_central_differences(orc, name):
    w, tl, g, phys, pos, csr, lap, u = _case(name)
    got = O.r2_dtheta(phys, w.vol, w.phi[0], g, w.kernel, w.R, w.mapspec, tl, csr)
    h = 1e-6
    fd = np.zeros(len(tl))
    for q, t in enumerate(tl):
        terms = [list(x) for x in w.mapspec.terms]
        sp, sm = I.MapSpec(**{**w.mapspec.__dict__}), I.MapSpec(**{**w.mapspec.__dict__})
        tp, tm = [list(x) for x in terms], [list(x) for x in terms]
        tp[t][0] += h
        tm[t][0] -= h
        sp.terms, sm.terms = [tuple(x) for x in tp], [tuple(x) for x in tm]
        a = O.sph2(O.project(phys, sp), w.vol, w.phi[0], w.kernel, w.R, sp, csr=csr)[0][:, 0, O.I_LAP]
        b = O.sph2(O.project(phys, sm), w.vol, w.phi[0], w.kernel, w.R, sm, csr=csr)[0][:, 0, O.I_LAP]
        fd[q] = np.sum((a - b) * (a + b - 2.0 * g)) / (2 * h)
    scale = np.abs(fd).max()
    err = np.abs(got - fd) / np.maximum(np.abs(fd), 1e-3 * scale)
    print(f"\n{name}: R2 dtheta vs central differences, worst relative {err.max():.1e}")
    assert err.max() <= 1e-5
    assert scale > 0


def test_dtheta_is_r1_plus_the_height_chain(orc):
    w, tl, g, phys, pos, csr, lap, u = _case("sigma3d")
    full = O.r2_dtheta(phys, w.vol, w.phi[0], g, w.kernel, w.R, w.mapspec, tl, csr)
    rec, _ = O.sph2(pos, w.vol, w.phi[0], w.kernel, w.R, w.mapspec, csr=csr)
    r1 = O.dtheta(pos, w.mapspec, u, rec[:, 0, O.I_DHAT], tl)
    gz = O.r2_dzhat(pos, w.vol, w.phi[0], w.kernel, w.R, w.mapspec, u, csr=csr)
    h = 1e-7
    chain = np.zeros(len(tl))
    for q, t in enumerate(tl):
        tp = [list(x) for x in w.mapspec.terms]
        tm = [list(x) for x in w.mapspec.terms]
        tp[t][0] += h
        tm[t][0] -= h
        sp = I.MapSpec(w.mapspec.kind, w.mapspec.Hhat, w.mapspec.H, w.mapspec.dmin, w.mapspec.eps,
                       [tuple(x) for x in tp])
        sm = I.MapSpec(w.mapspec.kind, w.mapspec.Hhat, w.mapspec.H, w.mapspec.dmin, w.mapspec.eps,
                       [tuple(x) for x in tm])
        dz = (O.project(phys, sp)[-1] - O.project(phys, sm)[-1]) / (2 * h)
        chain[q] = np.dot(gz, dz)
    tot = r1 + chain
    scale = np.abs(full).max()
    assert np.abs(tot - full).max() <= 1e-7 * scale
    # the height chain is not negligible: R1 alone is a different quantity
    assert np.abs(chain).max() > 1e-2 * scale


def test_translation_invariance_of_the_sph2_part(orc):
    w, tl, g, phys, pos, csr, lap, u = _case("sigma3d")
    gz = O.r2_dzhat(pos, w.vol, w.phi[0], w.kernel, w.R, w.mapspec, u, csr=csr, ct_dep=False)
    assert abs(gz.sum()) <= 1e-10 * np.abs(gz).sum()
    gz1 = O.r2_dzhat(pos, w.vol, w.phi[0], w.kernel, w.R, w.mapspec, u, csr=csr, ct_dep=True)
    assert abs(gz1.sum()) > 1e-6 * np.abs(gz1).sum()
