"""Pins of the oracle's pressure-step functions (Sec. 3.3, Eqs. VCT_ppe,
VCT_ppe_w, div_1st, gra_1st): the explicit Laplacian weights, the J-mapped
first-order divergence and pressure gradient, the projected-space density, the
right-hand side and the BiCGSTAB solve."""
import numpy as np
import pytest

from paper_2607_28872_amd import inputs as I
import oracle as O

from test_oracle import _fd_physical_derivatives, _map_values

FAMILIES = ["bf2d", "bfe2d", "sigma3d"]


def _phys_points(w):
    """Physical positions of the particles, (dim, n)."""
    d = w.dim
    y = w.pos[1] if d == 3 else None
    a, b = _map_values(w.mapspec, w.pos[0], y)
    zp = w.pos[d - 1] / a - b
    return np.stack(([w.pos[0], w.pos[1]] if d == 3 else [w.pos[0]]) + [zp])


def _projected(w, q):
    """Projected coordinates of physical points q (list of arrays)."""
    d = w.dim
    a, b = _map_values(w.mapspec, q[0], q[1] if d == 3 else None)
    return np.stack(list(q[: d - 1]) + [a * (q[d - 1] + b)])


@pytest.mark.parametrize("family", FAMILIES)
def test_laplacian_weights_reproduce_the_operator(orc, family):
    """sum_j W_ij (phi_j - phi_i) equals the oracle's Laplacian (Eq. lap_VCT)
    of both fields at every particle."""
    w = I.small(family)
    csr = O.neighbors(w.pos, w.R)
    wts, fl = O.lap_weights(w.pos, w.vol, w.kernel, w.R, w.mapspec, csr=csr)
    assert not fl.any()
    rec, _ = O.sph2(w.pos, w.vol, w.phi, w.kernel, w.R, w.mapspec, csr=csr)
    for f in range(w.phi.shape[0]):
        got = O.ppe_matvec(wts, None, w.phi[f])
        ref = rec[:, f, O.I_LAP]
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()


@pytest.mark.parametrize("family", FAMILIES)
def test_divergence_and_gradient_exact_for_projected_linear_fields(orc, family):
    """For fields linear in the projected coordinates the first-order gradients
    are exact (Eq. gra_1st), so the divergence of v and the corrector's
    pressure gradient equal their physical derivatives, here by fourth-order
    central differences in physical coordinates."""
    w = I.small(family)
    d = w.dim
    rng = np.random.default_rng(7)
    a = rng.uniform(-1, 1, d)
    B = rng.uniform(-1, 1, (d, d))
    c0, cg = rng.uniform(-1, 1), rng.uniform(-1, 1, d)
    v = a[:, None] + B @ w.pos
    p = c0 + cg @ w.pos
    csr = O.neighbors(w.pos, w.R)
    rho, dt = 1.3, 0.01
    rhs, div, dens = O.ppe_rhs(w.pos, w.vol, w.kernel, w.R, w.mapspec, v, rho, dt, 0.0, csr=csr)
    pp = _phys_points(w)
    div_fd = np.zeros(w.n)
    for I_ in range(d):
        g, _ = _fd_physical_derivatives(lambda q: a[I_] + B[I_] @ _projected(w, q), pp, 1e-4)
        div_fd += g[I_]
    assert np.abs(div - div_fd).max() <= 1e-7 * np.abs(div_fd).max()
    assert np.allclose(rhs, rho / dt * div, rtol=1e-14, atol=0)
    gp, _ = _fd_physical_derivatives(lambda q: c0 + cg @ _projected(w, q), pp, 1e-4)
    vstar = rng.uniform(-1, 1, (d, w.n))
    vout = O.ppe_correct(w.pos, w.vol, w.kernel, w.R, w.mapspec, p, vstar, rho, dt, csr=csr)
    assert np.abs(vout - (vstar - dt / rho * gp)).max() <= 1e-7 * dt / rho * np.abs(gp).max()


def test_density_is_the_kernel_sum(orc):
    """dens_i = rho (V_i w(0) + sum_{j in S_i} V_j w(r_ij)) against a numpy sum
    over all pairs, and close to rho in the interior of an unjittered lattice
    (the kernel's unit integral)."""
    w = I.small("sigma3d")
    rho = 0.9
    _, _, dens = O.ppe_rhs(w.pos, w.vol, w.kernel, w.R, w.mapspec, np.zeros_like(w.pos), rho, 1.0, 0.0)
    idx = np.arange(0, w.n, 97)
    dx = w.pos[:, idx, None] - w.pos[:, None, :]
    r = np.sqrt((dx * dx).sum(axis=0))
    q = r / w.R
    C = 21.0 / (2.0 * np.pi * w.R ** 3)
    wv = np.where(q < 1.0, C * (1 - q) ** 4 * (1 + 4 * q), 0.0)
    ref = rho * (wv * w.vol[None, :]).sum(axis=1)
    assert np.abs(dens[idx] - ref).max() <= 1e-13 * rho
    lat = I.make_sigma3d(24, 24, 24, 0.0, nx_span=24)
    _, _, dl = O.ppe_rhs(lat.pos, lat.vol, lat.kernel, lat.R, lat.mapspec, np.zeros_like(lat.pos), rho, 1.0, 0.0)
    inner = np.all((lat.pos > lat.R) & (lat.pos < np.asarray(lat.hi)[:, None] - lat.R), axis=0)
    assert np.abs(dl[inner] / rho - 1.0).max() < 2e-2


def test_rhs_terms_and_dirichlet_rows(orc):
    """rhs = rho/dt div + gamma (rho Jbar/J - dens)/dt^2 (Eq. VCT_ppe_w), the
    prescribed value on Dirichlet rows."""
    w = I.small("sigma3d")
    rng = np.random.default_rng(8)
    v = rng.uniform(-1, 1, w.pos.shape)
    jr = rng.uniform(0.9, 1.1, w.n)
    dirichlet = I.boundary_layer(w.pos, w.lo, w.hi, w.R)
    pbc = rng.uniform(-1, 1, w.n)
    rho, dt, gamma = 1.0, 1e-3, 1e-1
    rhs, div, dens = O.ppe_rhs(w.pos, w.vol, w.kernel, w.R, w.mapspec, v, rho, dt, gamma, jr=jr,
                               dirichlet=dirichlet, pbc=pbc)
    ref = rho / dt * div + gamma * (rho * jr - dens) / dt ** 2
    inner = ~dirichlet
    assert np.allclose(rhs[inner], ref[inner], rtol=1e-14, atol=0)
    assert np.array_equal(rhs[dirichlet], pbc[dirichlet])


def test_bicgstab_matches_a_direct_sparse_solve(orc):
    """The oracle's BiCGSTAB against scipy's sparse LU on the same system."""
    sp = pytest.importorskip("scipy.sparse")
    spl = pytest.importorskip("scipy.sparse.linalg")
    w = I.small("bf2d")
    wts, fl = O.lap_weights(w.pos, w.vol, w.kernel, w.R, w.mapspec)
    rp, col, W = wts
    dirichlet = I.boundary_layer(w.pos, w.lo, w.hi, w.R)
    n = w.n
    rows = np.repeat(np.arange(n), np.diff(rp))
    # A_ij = W_ij, A_ii = -sum_j W_ij on ordinary rows; identity rows for Dirichlet
    keep = ~dirichlet[rows]
    diag = np.where(dirichlet, 1.0, -np.bincount(rows, weights=W, minlength=n))
    A = sp.csc_matrix((np.concatenate([W[keep], diag]), (np.concatenate([rows[keep], np.arange(n)]),
                                                         np.concatenate([col[keep], np.arange(n)]))), shape=(n, n))
    b = np.random.default_rng(9).standard_normal(n)
    xd = spl.spsolve(A, b)
    x, it, rr, st = O.ppe_bicgstab(wts, dirichlet, b, tol=1e-13, maxit=5000)
    print(f"\nBiCGSTAB: {it} iterations, relres {rr:.1e}")
    # stopped on the recurrence residual (1e-13); the true residual trails it
    # by the rounding of the updates
    assert st == 0 and rr <= 1e-11
    assert np.abs(x - xd).max() <= 1e-9 * np.abs(xd).max()
    assert np.abs(O.ppe_matvec(wts, dirichlet, x) - A @ x).max() <= 1e-9 * np.abs(b).max()


@pytest.mark.parametrize("family", ["bfe2d", "sigma3d"])
def test_manufactured_pressure_is_recovered(orc, family):
    """p = P, a quadratic in projected coordinates: SPH(2) reproduces it, so
    the interior rows of A P equal the physical Laplacian of P (finite
    differences in physical coordinates) and the solve with that right-hand
    side and P on the Dirichlet rows returns P."""
    w = I.small(family)
    c = w.extra["pquad"]
    P = I.eval_quadratic(c, w.pos)
    wts, fl = O.lap_weights(w.pos, w.vol, w.kernel, w.R, w.mapspec)
    dirichlet = I.boundary_layer(w.pos, w.lo, w.hi, w.R)
    b = O.ppe_matvec(wts, dirichlet, P)
    _, H = _fd_physical_derivatives(lambda q: I.eval_quadratic(c, _projected(w, q)), _phys_points(w), 1e-4)
    lap_fd = np.trace(H)
    inner = ~dirichlet
    assert np.abs(b[inner] - lap_fd[inner]).max() <= 1e-6 * np.abs(lap_fd).max()
    x, it, rr, st = O.ppe_bicgstab(wts, dirichlet, b, tol=1e-13, maxit=5000)
    print(f"\n{family}: {it} iterations, relres {rr:.1e}")
    assert st == 0
    assert np.abs(x - P).max() <= 1e-9 * np.abs(P).max()
