"""Pins of the oracle's volume smoothing (Sec. 3.6, Eq. VCT_bar_a): the
smoothed Jacobian determinant Jbar^N of the sigma method, updated pair by pair
along the neighbours of each target particle.

What fixes it independently of the oracle's own formula:
  * the paper defines the update as a volume exchange, V'_i = V_i + dV_ij and
    V'_j = V_j - dV_ij with V_i = J_i / Jbar_i V; a plain Python loop in that
    volume form (not the closed form Eq. VCT_bar_a) must give the same Jbar;
  * the exchange conserves the total volume sum_i J_i / Jbar_i exactly;
  * two particles have a closed form (the volume difference shrinks by
    (1 - 2c) at each of the two visits, c = C_V (r_e - r) / r_e);
  * equal volume ratios are a fixed point; C_V = 0 changes nothing;
  * every update is a convex combination (c < 1), so the ratios stay within
    their initial range.
"""
import numpy as np
import pytest

from paper_2607_28872_amd import inputs as I
import oracle as O

CV = 1e-2        # C_V = dt x 10^2 with dt = 1e-4, the setting the paper adopts


def _sigma_set(nx=14, ny=12, nz=8, seed=0):
    w = I.make_sigma3d(nx, ny, nz, 0.05, seed=seed, name="jbar-small", nx_span=nx)
    J = O.alpha_beta(3, w.pos[0], w.pos[1], w.mapspec)[:, 0]
    return w, J


def _brute_csr(pos, R, rng=None):
    """Neighbour rows by brute force in numpy (columns in a random order per
    row when rng is given)."""
    d2 = ((pos[:, :, None] - pos[:, None, :]) ** 2).sum(axis=0)
    n = pos.shape[1]
    rows = []
    for i in range(n):
        js = np.nonzero((d2[i] < R * R) & (np.arange(n) != i))[0]
        if rng is not None:
            js = rng.permutation(js)
        rows.append(js)
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.concatenate(rows).astype(np.int32) if rp[-1] else np.zeros(0, np.int32)
    return rp, col


def _volume_form(pos, J, jbar, cv, re, order, csr):
    """The exchange written with volumes (the paper's dV_ij and V' = V +- dV),
    in units of the representative volume V."""
    rp, col = csr
    v = [J[i] / jbar[i] for i in range(len(J))]
    for i in order:
        for k in range(rp[i], rp[i + 1]):
            j = int(col[k])
            r = float(np.sqrt(((pos[:, j] - pos[:, i]) ** 2).sum()))
            dv = cv * (re - r) / re * (v[j] - v[i])
            v[i] = v[i] + dv
            v[j] = v[j] - dv
    return np.array([J[i] / v[i] for i in range(len(J))])


@pytest.mark.parametrize("dim", [2, 3])
def test_jbar_matches_the_volume_exchange(orc, dim):
    rng = np.random.default_rng(11)
    if dim == 2:
        w = I.make_2d(9, 7, 1.0, 0.10, name="jbar-2d")
        J = 1.0 + 0.3 * rng.uniform(size=w.n)          # any positive determinant
    else:
        w = I.make_sigma3d(7, 6, 5, 0.05, name="jbar-3d", nx_span=7)
        J = O.alpha_beta(3, w.pos[0], w.pos[1], w.mapspec)[:, 0]
    jb0 = J * I.volume_perturbation(w.n, amp=0.2)
    csr = _brute_csr(w.pos, w.R, rng)
    order = rng.permutation(w.n)
    cv = 0.3                                            # large, so every pair moves visibly
    got = O.jbar_smooth(w.pos, J, jb0, cv, w.R, order=order, csr=csr)
    ref = _volume_form(w.pos, J, jb0, cv, w.R, order, csr)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(got - jb0).max() > 1e-3 * np.abs(jb0).max()


def test_jbar_conserves_total_volume(orc):
    w, J = _sigma_set()
    jb0 = J * I.volume_perturbation(w.n)
    got = O.jbar_smooth(w.pos, J, jb0, CV, w.R)
    v0, v1 = np.sum(J / jb0), np.sum(J / got)
    assert abs(v1 - v0) <= 1e-13 * v0
    # the ratios moved towards each other
    assert np.std(J / got) < np.std(J / jb0)


def test_jbar_two_particles_closed_form(orc):
    R = 1.0
    pos = np.array([[0.0, 0.37], [0.0, 0.0]])
    J = np.array([2.0, 3.0])
    jb0 = np.array([1.7, 3.4])
    cv = 0.25
    got = O.jbar_smooth(pos, J, jb0, cv, R, order=[0, 1], csr=(np.array([0, 1, 2]), np.array([1, 0], np.int32)))
    v0, v1 = J / jb0
    c = cv * (R - 0.37) / R
    s, d = v0 + v1, (v1 - v0) * (1.0 - 2.0 * c) ** 2
    ref = J / np.array([(s - d) / 2.0, (s + d) / 2.0])
    assert np.abs(got - ref).max() <= 4e-16 * np.abs(ref).max()


def test_jbar_fixed_points(orc):
    w, J = _sigma_set(10, 9, 6)
    # equal ratios: nothing moves (up to the rounding of J Jbar / J)
    got = O.jbar_smooth(w.pos, J, J.copy(), CV, w.R)
    assert np.abs(got - J).max() <= 2.3e-16 * np.abs(J).max()
    # no smoothing
    jb0 = J * I.volume_perturbation(w.n)
    got = O.jbar_smooth(w.pos, J, jb0, 0.0, w.R)
    assert np.abs(got - jb0).max() <= 2.3e-16 * np.abs(jb0).max()


def test_jbar_stays_within_the_initial_range(orc):
    w, J = _sigma_set()
    jb0 = J * I.volume_perturbation(w.n, amp=0.3)
    got = O.jbar_smooth(w.pos, J, jb0, 0.4, w.R)
    r0, r1 = J / jb0, J / got
    assert r1.min() >= r0.min() * (1 - 1e-15) and r1.max() <= r0.max() * (1 + 1e-15)


def test_jbar_depends_on_the_visiting_order(orc):
    """The update is sequential: two visiting orders give different results
    (beyond rounding), each conserving the total volume."""
    w, J = _sigma_set(10, 9, 6)
    jb0 = J * I.volume_perturbation(w.n)
    a = O.jbar_smooth(w.pos, J, jb0, 0.2, w.R)
    b = O.jbar_smooth(w.pos, J, jb0, 0.2, w.R, order=np.arange(w.n)[::-1])
    assert np.abs(a - b).max() > 1e-6
    for x in (a, b):
        assert abs(np.sum(J / x) - np.sum(J / jb0)) <= 1e-13 * np.sum(J / jb0)
