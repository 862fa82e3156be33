"""Pins of the oracle's conventional ISPH operators (the ISPH case of Table
case_names): the 0th-order models of Sec. 3.1 (gradient, Espanol-Revenga
second derivatives of Eq. sec_0th, Brookshaw Laplacian) and the summation
pressure gradient of Eq. gra_sum.

These operators are not exact for polynomials on a finite particle set, so the
pins are the properties that hold without that:
  * the trace of the Eq. sec_0th Hessian is the Brookshaw Laplacian on any set
    (the weights sum to c - d = 2 in 2-D and 3-D), to rounding;
  * on a lattice with R / dx growing, the lattice sums tend to the kernel
    integrals, for which the 0th-order models are exact on quadratics: the
    errors shrink with R / dx and are small at R = 16 dx;
  * through a non-affine map the physical slots follow finite differences of
    the physical field at that resolution;
  * the summation gradient conserves momentum: sum_i V_i <grad^ p>^+_i = 0 for
    any particle set, pressures and densities (the pair terms are
    antisymmetric), to rounding;
  * a constant pressure on a centrally symmetric neighbourhood has zero
    summation gradient.
"""
import numpy as np
import pytest

import oracle as O
from paper_2607_28872_amd import inputs as I
from test_oracle import _fd_physical_derivatives, _map_values

IDENT = I.MapSpec(I.MAP_IDENTITY, 1.0, 1.0, 0.0, 0.0, [])


def _proj_hessian(rec, dim):
    """Projected Hessian (dim x dim) from the D^ slots and the doubled-cross D slots."""
    dh = rec[O.I_DHAT]
    H = np.zeros((3, 3))
    H[0, 0], H[1, 1], H[2, 2] = dh[1], dh[2], dh[3]
    H[0, 2] = H[2, 0] = dh[4]
    H[1, 2] = H[2, 1] = dh[5]
    H[0, 1] = H[1, 0] = 0.5 * rec[O.I_D][3] if dim == 3 else 0.0
    ax = [0, 1, 2] if dim == 3 else [0, 2]
    return H[np.ix_(ax, ax)]


def _centred_lattice(dim, h, dx=1.0 / 64, centre=None):
    k = h + 1
    ax = np.arange(-k, k + 1) * dx
    grids = np.meshgrid(*([ax] * dim), indexing="ij")
    pos = np.stack([g.ravel() for g in grids])
    c = int(np.argmin((pos ** 2).sum(0)))
    if centre is not None:
        pos = pos + np.asarray(centre, dtype=float)[:, None]
    return pos, c, np.full(pos.shape[1], dx ** dim), h * dx


@pytest.mark.parametrize("family", ["bf2d", "sigma3d"])
def test_sec0th_trace_is_the_brookshaw_laplacian(family):
    w = I.small(family)
    rows = np.arange(0, w.n, 7)
    phi = np.vstack([w.phi, np.random.default_rng(3).uniform(-1, 1, w.n)])
    out, fl = O.ops0(w.pos, w.vol, phi, w.kernel, w.R, IDENT, rows=rows)
    assert not fl.any()
    tr = out[:, :, O.I_DHAT][:, :, 1:4].sum(-1)
    lb = O.lap0(w.pos, w.vol, phi, w.kernel, w.R, rows=rows)
    err = np.abs(tr - lb).max() / np.abs(lb).max()
    print(f"\n{family}: |trace(H0) - Brookshaw| / max = {err:.1e}")
    assert err <= 1e-13
    # under the identity map the physical Laplacian is that same trace
    assert np.abs(out[:, :, O.I_LAP] - lb).max() <= 1e-13 * np.abs(lb).max()


@pytest.mark.parametrize("family", ["bf2d", "sigma3d"])
def test_record_slots_follow_the_record_layout(family):
    """The D slots (xx, yy, zz, 2xy, 2xz, 2yz) and the D^ slots
    (dz^, xx, yy, zz, xz, yz) hold the same second derivatives, the gradient
    slots the same gradient, and 2-D records leave every y slot zero."""
    w = I.small(family)
    out, _ = O.ops0(w.pos, w.vol, w.phi, w.kernel, w.R, w.mapspec, rows=np.arange(0, w.n, 11))
    r = out.reshape(-1, O.REC)
    D, Dh = r[:, O.I_D], r[:, O.I_DHAT]
    assert np.array_equal(D[:, 0], Dh[:, 1]) and np.array_equal(D[:, 1], Dh[:, 2])
    assert np.array_equal(D[:, 2], Dh[:, 3])
    assert np.array_equal(D[:, 4], 2 * Dh[:, 4]) and np.array_equal(D[:, 5], 2 * Dh[:, 5])
    assert np.array_equal(r[:, O.I_G1], r[:, O.I_G2]) and np.array_equal(r[:, O.I_G1][:, 2], Dh[:, 0])
    if w.dim == 2:
        y = [1, 4, 6, 8, 10, 12, 14, 17, 20, 22, 24, 27, 30]
        assert not r[:, y].any()


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("kernel", [I.KERNEL_WENDLAND_C2, I.KERNEL_CUBIC_SPLINE])
def test_zeroth_order_models_tend_to_the_exact_derivatives(dim, kernel):
    rng = np.random.default_rng(11 + dim)
    H = rng.uniform(-1, 1, (dim, dim))
    H = H + H.T
    g = rng.uniform(-1, 1, dim)
    errs = {}
    for h in (8, 16):
        pos, c, vol, R = _centred_lattice(dim, h)
        phi = 0.5 * np.einsum("an,ab,bn->n", pos, H, pos) + g @ pos + 0.3
        out, fl = O.ops0(pos, vol, phi, kernel, R, IDENT, rows=[c])
        assert not fl.any()
        rec = out[0, 0]
        ax = [0, 1, 2] if dim == 3 else [0, 2]
        eg = np.abs(rec[O.I_G1][ax] - g).max() / np.abs(g).max()
        eh = np.abs(_proj_hessian(rec, dim) - H).max() / np.abs(H).max()
        el = abs(O.lap0(pos, vol, phi, kernel, R, rows=[c])[0, 0] - np.trace(H)) / np.abs(H).max()
        errs[h] = (eg, eh, el)
    print(f"\n{dim}-D kernel {kernel}: (grad, hessian, brookshaw) errors by R/dx", errs)
    eg, eh, el = errs[16]
    assert eg <= 1e-5 and el <= 1e-5 and eh <= 1e-3
    assert errs[16][1] < errs[8][1]


@pytest.mark.parametrize("family", ["bf2d", "sigma3d"])
def test_zeroth_order_physical_slots_follow_finite_differences(family):
    """A projected quadratic on a fine lattice (R = 16 dx) placed inside the
    mapped domain: the physical slots against fourth-order differences of
    phi(x, y, z) = P(x, y, alpha (z + beta)) in physical coordinates."""
    w = I.small(family)
    d, ms = w.dim, w.mapspec
    centre = [0.37, 0.41, 0.5 * w.hi[2]] if d == 3 else [0.37, 0.5 * w.hi[1]]
    pos, c, vol, R = _centred_lattice(d, 16, dx=1.0 / 2048, centre=centre)
    cq = np.random.default_rng(17).uniform(-1, 1, 10 if d == 3 else 6)
    phi = I.eval_quadratic(cq, pos)
    out, fl = O.ops0(pos, vol, phi, w.kernel, R, ms, rows=[c])
    assert not fl.any()
    rec = out[0, 0]
    p = pos[:, c:c + 1]
    x, y = p[0], (p[1] if d == 3 else None)
    a, b = _map_values(ms, x, y)
    pphys = np.stack(([x, p[1]] if d == 3 else [x]) + [p[d - 1] / a - b])

    def phi_phys(q):
        aa, bb = _map_values(ms, q[0], q[1] if d == 3 else None)
        return I.eval_quadratic(cq, np.stack(list(q[:d - 1]) + [aa * (q[d - 1] + bb)]))

    g_fd, H_fd = _fd_physical_derivatives(phi_phys, pphys, 1e-4)
    g_fd, H_fd = g_fd[:, 0], H_fd[:, :, 0]
    ax = [0, 1, 2] if d == 3 else [0, 2]
    got_g = rec[O.I_GRAD][ax]
    hess_slot = {(0, 0): 7, (1, 1): 8, (2, 2): 9, (0, 1): 10, (0, 2): 11, (1, 2): 12}
    got_H = np.array([[rec[hess_slot[tuple(sorted((ax[i], ax[j])))]] for j in range(d)] for i in range(d)])
    eg = np.abs(got_g - g_fd).max() / np.abs(g_fd).max()
    eh = np.abs(got_H - H_fd).max() / np.abs(H_fd).max()
    el = abs(rec[O.I_LAP] - np.trace(H_fd)) / np.abs(H_fd).max()
    # the curvature term phi_z^ grad grad z^ is large against the bar
    mev = O.map_eval(d, x, y, p[d - 1], ms)
    curv = np.abs(rec[O.I_G1][2] * mev[0, 15:]).max()
    print(f"\n{family}: physical errors grad {eg:.1e} hessian {eh:.1e} laplacian {el:.1e}; "
          f"curvature term / max |H| = {curv / np.abs(H_fd).max():.1e}")
    assert eg <= 1e-4 and eh <= 2e-3 and el <= 2e-3
    assert curv > 20 * 2e-3 * np.abs(H_fd).max()


@pytest.mark.parametrize("family", ["bf2d", "sigma3d"])
def test_summation_gradient_conserves_momentum(family):
    w = I.small(family)
    rng = np.random.default_rng(23)
    p = rng.uniform(-1, 1, w.n)
    rho = rng.uniform(0.8, 1.25, w.n)
    _, gh, fl = O.grad_sum(w.pos, w.vol, p, w.kernel, w.R, w.mapspec, rho=rho)
    assert not fl.any()
    tot = (w.vol[:, None] * gh).sum(0)
    scale = np.abs(w.vol[:, None] * gh).sum(0).max()
    print(f"\n{family}: |sum_i V_i grad^ p_i| / sum |.| = {np.abs(tot).max() / scale:.1e}")
    assert np.abs(tot).max() <= 1e-13 * scale


def test_summation_gradient_of_a_constant_on_a_symmetric_set_is_zero():
    pos, c, vol, R = _centred_lattice(3, 3)
    p = np.full(pos.shape[1], 2.5)
    _, gh, fl = O.grad_sum(pos, vol, p, I.KERNEL_WENDLAND_C2, R, IDENT, rows=[c])
    # each of the pair terms is about 2 p V |grad w| ~ 1e2 here
    assert np.abs(gh).max() <= 1e-11


@pytest.mark.parametrize("dim", [2, 3])
def test_summation_gradient_tends_to_the_exact_gradient(dim):
    g = np.array([0.7, -0.4, 1.1])[:dim]
    errs = []
    for h in (8, 16):
        pos, c, vol, R = _centred_lattice(dim, h)
        p = g @ pos + 0.25
        ph, gh, fl = O.grad_sum(pos, vol, p, I.KERNEL_WENDLAND_C2, R, IDENT, rows=[c], rho0=1.3)
        ax = [0, 1, 2] if dim == 3 else [0, 2]
        errs.append(np.abs(gh[0, ax] - g).max() / np.abs(g).max())
        assert np.array_equal(ph[0], gh[0]) or np.abs(ph[0] - gh[0]).max() <= 1e-15
    print(f"\n{dim}-D summation gradient errors at R/dx = 8, 16: {errs}")
    assert errs[1] <= 1e-5 and errs[1] < errs[0]
