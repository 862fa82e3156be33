"""Pins of the oracle's per-particle mapping kind: alpha, beta and their
first and second horizontal derivatives given at every particle (Sec. 2.1,
Eq. VCT, for a measured or tabulated bottom).

  * a table filled with the values of the bottom-defined maps (BF, BFE,
    sigma) gives the same records, bit for bit, as those maps;
  * a transformation that no bottom-term kind can express (alpha and beta
    varying independently in x and y, written out here with their
    derivatives) carries exact projected derivatives of a projected quadratic
    to the physical derivatives of phi(x, y, z) = P(x, y, alpha (z + beta)),
    taken by finite differences in physical coordinates: gradient,
    Laplacian, Hessian, cross derivatives and the trace.
"""
import numpy as np
import pytest

from paper_2607_28872_amd import inputs as I
import oracle as O

from test_oracle import _fd_physical_derivatives


def _table(w):
    return np.ascontiguousarray(O.alpha_beta(w.dim, w.pos[0], w.pos[1] if w.dim == 3 else None, w.mapspec).T)


@pytest.mark.parametrize("family", ["bf2d", "bfe2d", "sigma3d"])
def test_table_of_a_bottom_map_gives_its_records(orc, family):
    w = I.small(family)
    pp = I.MapSpec(kind=I.MAP_PER_PARTICLE, pp=_table(w))
    csr = O.neighbors(w.pos, w.R)
    a, fa = O.sph2(w.pos, w.vol, w.phi, w.kernel, w.R, w.mapspec, csr=csr)
    b, fb = O.sph2(w.pos, w.vol, w.phi, w.kernel, w.R, pp, csr=csr)
    assert np.array_equal(fa, fb)
    assert np.array_equal(a, b)
    a0, _ = O.ops0(w.pos, w.vol, w.phi, w.kernel, w.R, w.mapspec, csr=csr)
    b0, _ = O.ops0(w.pos, w.vol, w.phi, w.kernel, w.R, pp, csr=csr)
    assert np.array_equal(a0, b0)


# a transformation of the form of Eq. VCT beyond the bottom-term kinds
K = 2 * np.pi


def _ab(x, y):
    """alpha, beta and derivatives [a, ax, ay, axx, axy, ayy, b, bx, by, bxx, bxy, byy]."""
    a = 1.2 + 0.2 * np.sin(K * x) * np.cos(K * y)
    ax = 0.2 * K * np.cos(K * x) * np.cos(K * y)
    ay = -0.2 * K * np.sin(K * x) * np.sin(K * y)
    axx = -0.2 * K * K * np.sin(K * x) * np.cos(K * y)
    axy = -0.2 * K * K * np.cos(K * x) * np.sin(K * y)
    ayy = -0.2 * K * K * np.sin(K * x) * np.cos(K * y)
    b = 0.1 * np.cos(K * x) + 0.05 * np.sin(K * y) + 0.03 * x * y
    bx = -0.1 * K * np.sin(K * x) + 0.03 * y
    by = 0.05 * K * np.cos(K * y) + 0.03 * x
    bxx = -0.1 * K * K * np.cos(K * x)
    bxy = 0.03 + 0.0 * x
    byy = -0.05 * K * K * np.sin(K * y)
    return np.stack([a, ax, ay, axx, axy, ayy, b, bx, by, bxx, bxy, byy])


def test_tabulated_map_chain_rule(orc):
    w = I.small("sigma3d")
    c = w.extra["pquad"]
    x, y = w.pos[0], w.pos[1]
    tab = _ab(x, y)
    ms = I.MapSpec(kind=I.MAP_PER_PARTICLE, pp=tab)
    zp = w.pos[2] / tab[0] - tab[6]

    def phi_phys(q):
        t = _ab(q[0], q[1])
        return I.eval_quadratic(c, np.stack([q[0], q[1], t[0] * (q[2] + t[6])]))

    g_fd, H_fd = _fd_physical_derivatives(phi_phys, np.stack([x, y, zp]), 1e-4)
    out, fl = orc.sph2(w.pos, w.vol, I.eval_quadratic(c, w.pos), w.kernel, w.R, ms)
    assert not fl.any()
    rec = out[:, 0]
    checks = {"lap": (rec[:, O.I_LAP], np.trace(H_fd)), "trace": (rec[:, O.I_LAP_TRACE], np.trace(H_fd))}
    for k in range(3):
        checks[f"grad{k}"] = (rec[:, k], g_fd[k])
    hess_slot = {(0, 0): 7, (1, 1): 8, (2, 2): 9, (0, 1): 10, (0, 2): 11, (1, 2): 12}
    for (p, q), s in hess_slot.items():
        checks[f"H{p}{q}"] = (rec[:, s], H_fd[p, q])
    tol = 1e-6
    worst = {}
    for nm, (got, ref) in checks.items():
        sc = np.abs(ref).max()
        assert sc > 1e3 * tol * np.abs(g_fd).max(), f"{nm} is too small to discriminate"
        worst[nm] = np.abs(got - ref).max() / sc
    print("\ntabulated map, physical slots vs finite differences:", {k: float(f"{v:.1e}") for k, v in worst.items()})
    assert max(worst.values()) <= tol, worst
