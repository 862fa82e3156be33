"""Seeded synthetic particle sets for the VCT-SPH(2) operator path.

This module only *describes* workloads: lattice positions in the projected
space, jitter, representative volumes, the bathymetry that defines a vertical
coordinate transformation (as plain coefficient data), and test fields.  It
evaluates none of the method's arithmetic (no neighbour search, no kernel, no
moment matrix, no Jacobian or Laplacian coefficient).  The GPU library and the
CPU oracle each turn the mapping descriptor into alpha/beta and their
derivatives with their own code.

Geometry conventions (paper Sec. 2.1, Eq. VCT):
  * 2-D sets use the vertical plane (x, z); 3-D sets use (x, y, z).
  * positions are given in the projected space r^ = (x, [y], z^) on a lattice
    of cell-centred points (i + 1/2) * dx with i.i.d. uniform jitter
    U(-j, j) * dx per coordinate, isotropic spacing dx in every direction.
  * representative volume V = dx**dim for every particle.
  * the bottom elevation h(x, y) is a sum of separable terms
    coef * B(x) * B(y) with B in {1, s, cos(2 pi f s), sin(2 pi f s)}.

Physical vertical positions are needed only to evaluate test fields defined
in physical coordinates (the 2-D sets).  For those sets the mapping has a
constant vertical scale a0 and beta = -h, so a particle at projected height
z^ sits at physical height z = h(x) + z^ / a0; that is the statement of where
the synthetic particles are, written out once here.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# basis kinds of one separable bathymetry factor
B_ONE, B_LIN, B_COS, B_SIN = 0, 1, 2, 3

# mapping kinds (paper Sec. 2.2)
MAP_IDENTITY, MAP_E, MAP_BF, MAP_BFE, MAP_SIGMA, MAP_PER_PARTICLE = 0, 1, 2, 3, 4, 5
MAP_NAMES = {MAP_IDENTITY: "identity", MAP_E: "E-SPH", MAP_BF: "BF-SPH",
             MAP_BFE: "BFE-SPH", MAP_SIGMA: "sigma-SPH", MAP_PER_PARTICLE: "per-particle"}

KERNEL_WENDLAND_C2, KERNEL_CUBIC_SPLINE = 0, 1

SEED_POS, SEED_QUAD, SEED_PQUAD, SEED_THETA, SEED_TARGET, SEED_ORDER, SEED_JBAR = 0, 1, 2, 3, 4, 5, 6


@dataclass
class MapSpec:
    """Plain-data description of a vertical coordinate transformation.

    kind   : MAP_* constant
    Hhat, H: projected / physical reference heights (E and BFE: alpha = Hhat/H;
             sigma: alpha = Hhat/(H - h))
    dmin, eps: sigma-SPH depth limiter, D_eff = smooth max(H - h, dmin; eps)
    terms  : list of (coef, bx, fx, by, fy) giving h = sum coef*Bx(x)*By(y)
    pp     : MAP_PER_PARTICLE only: (12, n) alpha, alpha_x, alpha_y, alpha_xx,
             alpha_xy, alpha_yy, beta, beta_x, beta_y, beta_xx, beta_xy,
             beta_yy at every particle (the particles' order)
    """
    kind: int = MAP_IDENTITY
    Hhat: float = 1.0
    H: float = 1.0
    dmin: float = 0.0
    eps: float = 0.0
    terms: list = field(default_factory=list)
    pp: object = None

    def with_terms(self, extra):
        return MapSpec(self.kind, self.Hhat, self.H, self.dmin, self.eps,
                       list(self.terms) + list(extra), self.pp)

    def as_array(self):
        """Terms as an (nterms, 5) float64 array: coef, bx, fx, by, fy."""
        if not self.terms:
            return np.zeros((0, 5), dtype=np.float64)
        return np.asarray(self.terms, dtype=np.float64).reshape(-1, 5)


@dataclass
class Workload:
    name: str
    dim: int
    counts: tuple            # lattice points per axis (x, [y], z)
    dx: float
    lo: tuple
    hi: tuple
    jitter: float
    kernel: int
    R: float
    mapspec: MapSpec
    pos: np.ndarray          # (dim, N) float64, projected coordinates
    vol: np.ndarray          # (N,) float64
    phi: np.ndarray          # (nf, N) float64
    field_names: list
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.pos.shape[1])


def basis(kind: int, freq: float, s: np.ndarray) -> np.ndarray:
    if kind == B_ONE:
        return np.ones_like(s)
    if kind == B_LIN:
        return s.copy()
    if kind == B_COS:
        return np.cos(2.0 * math.pi * freq * s)
    if kind == B_SIN:
        return np.sin(2.0 * math.pi * freq * s)
    raise ValueError(kind)


def bottom(terms, x: np.ndarray, y: np.ndarray | None = None) -> np.ndarray:
    """Bottom elevation h(x, y) of a term list (the workload's geometry)."""
    y = np.zeros_like(x) if y is None else y
    h = np.zeros_like(x)
    for coef, bx, fx, by, fy in terms:
        h = h + coef * basis(int(bx), fx, x) * basis(int(by), fy, y)
    return h


def lattice(counts, dx, jitter, seed=SEED_POS, shuffle=True, origin=None):
    """Jittered cell-centred lattice, returned as (dim, N) float64.

    The particle order is a seeded random permutation of the lattice order
    (shuffle=True) so that the library's cell sort has real work to do.
    """
    dim = len(counts)
    rng = np.random.default_rng(seed)
    axes = [(np.arange(c, dtype=np.float64) + 0.5) * dx for c in counts]
    grids = np.meshgrid(*axes, indexing="ij")
    pos = np.stack([g.reshape(-1) for g in grids])
    if origin is not None:
        pos = pos + np.asarray(origin, dtype=np.float64)[:, None]
    if jitter > 0:
        pos = pos + rng.uniform(-jitter, jitter, size=pos.shape) * dx
    if shuffle:
        order = np.random.default_rng(SEED_ORDER + seed * 1000).permutation(pos.shape[1])
        pos = np.ascontiguousarray(pos[:, order])
    return np.ascontiguousarray(pos)


def random_quadratic(dim, seed):
    """Coefficients (U[-1,1]) of a full quadratic polynomial in dim variables,
    ordered as [1, x_0..x_{d-1}, x_a*x_b for a<=b]."""
    nmono = 1 + dim + dim * (dim + 1) // 2
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=nmono)


def eval_quadratic(coef, coords):
    """Evaluate a quadratic given by random_quadratic() at coords (dim, N)."""
    dim = coords.shape[0]
    out = np.full(coords.shape[1], coef[0])
    k = 1
    for a in range(dim):
        out = out + coef[k] * coords[a]
        k += 1
    for a in range(dim):
        for b in range(a, dim):
            out = out + coef[k] * coords[a] * coords[b]
            k += 1
    return out


# ---------------------------------------------------------------------------
# workload families
# ---------------------------------------------------------------------------

def bf_bottom_terms():
    """b(x) = 0.2 + 0.1 sin(2 pi x)."""
    return [(0.2, B_ONE, 0.0, B_ONE, 0.0), (0.1, B_SIN, 1.0, B_ONE, 0.0)]


def sigma_bottom_terms():
    """Sloped beach: depth d = 1 - 0.95 x + 0.05 cos(2 pi y) with the still
    surface at H = 0, i.e. bottom elevation h = -d."""
    return [(-1.0, B_ONE, 0.0, B_ONE, 0.0), (0.95, B_LIN, 0.0, B_ONE, 0.0),
            (-0.05, B_ONE, 0.0, B_COS, 1.0)]


THETA_BASIS = [(B_ONE, 0.0), (B_COS, 1.0), (B_SIN, 1.0), (B_COS, 2.0)]


def theta_terms(theta):
    """16 Fourier-type perturbation terms theta_mn * c_m(x) * c_n(y)."""
    theta = np.asarray(theta, dtype=np.float64).reshape(4, 4)
    out = []
    for m, (bx, fx) in enumerate(THETA_BASIS):
        for n_, (by, fy) in enumerate(THETA_BASIS):
            out.append((float(theta[m, n_]), bx, fx, by, fy))
    return out


def make_2d(nx, nz, alpha0, jitter, seed=SEED_POS, kernel=KERNEL_WENDLAND_C2,
            name="2d", shuffle=True, kind=None):
    """2-D vertical-plane set over the projected box [0, nx dx) x [0, nz dx)
    with dx = 1/nx.  alpha0 = 1 gives BF-SPH, alpha0 != 1 gives BFE-SPH,
    both with the bottom b(x) = 0.2 + 0.1 sin(2 pi x)."""
    dx = 1.0 / nx
    pos = lattice((nx, nz), dx, jitter, seed, shuffle)
    terms = bf_bottom_terms()
    if kind is None:
        kind = MAP_BF if alpha0 == 1.0 else MAP_BFE
    ms = MapSpec(kind=kind, Hhat=float(alpha0), H=1.0, terms=terms)
    x, zh = pos
    zphys = bottom(terms, x) + zh / alpha0
    f_smooth = np.sin(2 * math.pi * x) * np.cos(math.pi * zphys)
    quad = random_quadratic(2, SEED_QUAD)
    f_main = f_smooth + eval_quadratic(quad, np.stack([x, zphys]))
    pquad = random_quadratic(2, SEED_PQUAD)
    f_exact = eval_quadratic(pquad, pos)
    R = 3.0 * dx if kernel == KERNEL_WENDLAND_C2 else 2.4 * dx
    return Workload(name=name, dim=2, counts=(nx, nz), dx=dx, lo=(0.0, 0.0),
                    hi=(nx * dx, nz * dx), jitter=jitter, kernel=kernel, R=R,
                    mapspec=ms, pos=pos, vol=np.full(pos.shape[1], dx * dx),
                    phi=np.ascontiguousarray(np.stack([f_main, f_exact])),
                    field_names=["f", "pquad"],
                    extra={"quad": quad, "pquad": pquad, "zphys": zphys})


def make_sigma3d(nx, ny, nz, jitter, seed=SEED_POS, kernel=KERNEL_WENDLAND_C2,
                 name="sigma3d", shuffle=True, theta=None, dmin=0.125, eps=0.01,
                 nx_span=None):
    """3-D sigma-SPH set: projected box [0,1)^2 x [0, Hhat), dx = 1/nx,
    Hhat = nz*dx, sloped-beach depth 1 -> 0.05 in x with a cos(2 pi y) ripple.
    nx_span lets a small test set cover a sub-range of the full domain."""
    dx = 1.0 / (nx if nx_span is None else nx_span)
    pos = lattice((nx, ny, nz), dx, jitter, seed, shuffle)
    Hhat = nz * dx
    terms = sigma_bottom_terms()
    if theta is not None:
        terms = terms + theta_terms(theta)
    ms = MapSpec(kind=MAP_SIGMA, Hhat=Hhat, H=0.0, dmin=dmin, eps=eps, terms=terms)
    x, y, zh = pos
    sig = zh / Hhat
    f_smooth = np.sin(2 * math.pi * x) * np.sin(2 * math.pi * y) * np.cos(math.pi * sig)
    quad = random_quadratic(3, SEED_QUAD)
    f_main = f_smooth + eval_quadratic(quad, pos)
    pquad = random_quadratic(3, SEED_PQUAD)
    f_exact = eval_quadratic(pquad, pos)
    R = 3.0 * dx if kernel == KERNEL_WENDLAND_C2 else 2.4 * dx
    return Workload(name=name, dim=3, counts=(nx, ny, nz), dx=dx, lo=(0.0, 0.0, 0.0),
                    hi=(nx * dx, ny * dx, Hhat), jitter=jitter, kernel=kernel, R=R,
                    mapspec=ms, pos=pos, vol=np.full(pos.shape[1], dx ** 3),
                    phi=np.ascontiguousarray(np.stack([f_main, f_exact])),
                    field_names=["f", "pquad"],
                    extra={"quad": quad, "pquad": pquad, "sigma": sig})


def target_field(pos, Hhat, scale=100.0, seed=SEED_TARGET, nmodes=8):
    """Seeded smooth target g for the Laplacian loss: nmodes products
    sin(2 pi (kx x + ky y) + p) cos(pi ks sigma), k in {0,1,2}, with a fixed
    RMS of `scale`."""
    rng = np.random.default_rng(seed)
    x, y, zh = pos
    sig = zh / Hhat
    g = np.zeros(pos.shape[1])
    for _ in range(nmodes):
        kx, ky, ks = rng.integers(0, 3, size=3)
        ph = rng.uniform(0, 2 * math.pi)
        amp = rng.uniform(-1, 1)
        g = g + amp * np.sin(2 * math.pi * (kx * x + ky * y) + ph) * np.cos(math.pi * ks * sig)
    rms = float(np.sqrt(np.mean(g * g))) if g.size else 1.0
    return g * (scale / (rms if rms > 0 else 1.0))


def boundary_layer(pos, lo, hi, width):
    """Particles within `width` of a face of the box [lo, hi) (bool, n): the
    Dirichlet rows of the synthetic pressure problems."""
    pos = np.asarray(pos)
    lo = np.asarray(lo, dtype=np.float64)[:, None]
    hi = np.asarray(hi, dtype=np.float64)[:, None]
    return np.any((pos < lo + width) | (pos >= hi - width), axis=0)


def velocity_field(pos):
    """A smooth seeded-free test velocity (dim, n) for the pressure step:
    v_I = sin(2 pi x + I) cos(pi z / z_max) + 0.1 (I + 1)."""
    pos = np.asarray(pos)
    zmax = float(pos[-1].max()) if pos.size else 1.0
    return np.stack([np.sin(2 * math.pi * pos[0] + a) * np.cos(math.pi * pos[-1] / zmax) + 0.1 * (a + 1)
                     for a in range(pos.shape[0])])


def volume_perturbation(n, amp=0.05, seed=SEED_JBAR):
    """Seeded factors 1 + U(-amp, amp) (n,): multiplied into the Jacobian
    determinant they give a previous smoothed determinant Jbar^(N-1) whose
    volume ratios J / Jbar scatter by about amp, as after particle motion."""
    return 1.0 + np.random.default_rng(seed).uniform(-amp, amp, size=n)


def theta0(seed=SEED_THETA):
    return np.random.default_rng(seed).uniform(-0.01, 0.01, size=16)


# ---------------------------------------------------------------------------
# the five named workloads and small same-shaped test sets
# ---------------------------------------------------------------------------

def config(name: str) -> Workload:
    """Named synthetic workloads.

    c0  2-D BF-SPH, 64x64 lattice (4,096), 10% jitter, alpha = 1.
    c1  2-D BFE-SPH, 2048x512 (1,048,576), alpha = 4, 10% jitter.
    c2  3-D sigma-SPH, 256x256x32 (2,097,152), 5% jitter.
    c3  3-D sigma-SPH, 512x512x32 (8,388,608), 5% jitter.
    c4  c2's particle set with 16 bathymetry perturbation coefficients.
    """
    if name == "c0":
        return make_2d(64, 64, 1.0, 0.10, name="c0")
    if name == "c1":
        return make_2d(2048, 512, 4.0, 0.10, name="c1")
    if name == "c2":
        return make_sigma3d(256, 256, 32, 0.05, name="c2")
    if name == "c3":
        return make_sigma3d(512, 512, 32, 0.05, name="c3")
    if name == "c4":
        w = make_sigma3d(256, 256, 32, 0.05, name="c4", theta=theta0())
        w.extra["theta"] = theta0()
        w.extra["target"] = target_field(w.pos, w.mapspec.Hhat)
        return w
    raise KeyError(name)


def small(family: str, seed=SEED_POS) -> Workload:
    """Small sets of each family, sized for the oracle to finish in seconds
    while spanning several GPU tiles and a ragged tail."""
    if family == "bf2d":
        return make_2d(72, 56, 1.0, 0.10, seed=seed, name="bf2d-small")
    if family == "bfe2d":
        return make_2d(96, 26, 4.0, 0.10, seed=seed, name="bfe2d-small")
    if family == "sigma3d":
        return make_sigma3d(30, 28, 12, 0.05, seed=seed, name="sigma3d-small", nx_span=30)
    if family == "sigma3d-adj":
        w = make_sigma3d(22, 20, 10, 0.05, seed=seed, name="sigma3d-adj", theta=theta0(), nx_span=22)
        w.extra["theta"] = theta0()
        w.extra["target"] = target_field(w.pos, w.mapspec.Hhat)
        return w
    raise KeyError(family)
