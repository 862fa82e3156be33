"""Adjoint of the Laplacian loss on the full 2.1M-particle sigma-SPH set with 16
bathymetry coefficients, through the torch.autograd bridge.

  * backward with the state recomputed, or solved again from the kept moment
    sums, equals backward with the state kept, bit for bit (the same kernels
    on the same inputs);
  * d/dphi along a seeded direction and d/dtheta for each coefficient against
    central differences with step 1e-6, within 1e-6 relative.  The loss is
    quadratic in phi, and the difference of squares is formed as
    (a - b)(a + b - 2 g), so the central difference is exact up to rounding;
  * d/dphi at sampled particles against the FP64 oracle's adjoint, with the
    oracle's own Laplacian (its u) on the rows the sampled entries need.
"""
import numpy as np
import pytest

import oracle as O
from paper_2607_28872_amd import inputs as I
from paper_2607_28872_amd import vct

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FD_STEP = 1e-6
FD_TOL = 1e-6


@pytest.fixture(scope="module")
def c4():
    from paper_2607_28872_amd.autograd import VctLaplacian, laplacian_loss
    w = I.config("c4")
    g = vct.Geometry(w.pos, w.vol, w.lo, w.hi, w.R, w.kernel, device=DEV, keep_col=True)
    ms = w.mapspec
    base = I.MapSpec(ms.kind, ms.Hhat, ms.H, ms.dmin, ms.eps, list(ms.terms[:-16]))
    phi = g.sorted_field(w.phi[0])[0]
    target = g.sorted_field(w.extra["target"])[0]
    theta = torch.tensor(w.extra["theta"].reshape(4, 4), dtype=torch.float64)
    return dict(w=w, g=g, base=base, phi=phi, target=target, theta=theta, Lap=VctLaplacian, loss=laplacian_loss)


def _grads(c, recompute):
    p = c["phi"].clone().requires_grad_(True)
    th = c["theta"].clone().requires_grad_(True)
    loss = c["loss"](c["g"], p, th, c["base"], c["target"], recompute)
    loss.backward()
    return p.grad.detach().clone(), th.grad.detach().clone()


def _lap(c, phi, theta):
    with torch.no_grad():
        return c["Lap"].apply(phi, theta, c["g"], c["base"], True)


def _dloss(c, lp, lm):
    """(L(+) - L(-)) for L = sum (lap - g)^2, as sum (lp - lm)(lp + lm - 2 g)."""
    return float(((lp - lm) * (lp + lm - 2.0 * c["target"])).sum())


def test_recomputed_state_gives_the_same_bits(c4):
    gp1, gt1 = _grads(c4, True)
    gp2, gt2 = _grads(c4, False)
    assert torch.equal(gp1, gp2)
    assert torch.equal(gt1, gt2)


def test_resolved_state_gives_the_same_bits(c4):
    """Backward from the kept moment sums (solve only) equals backward with
    the whole state recomputed."""
    gp1, gt1 = _grads(c4, True)
    gp2, gt2 = _grads(c4, "solve")
    assert torch.equal(gp1, gp2)
    assert torch.equal(gt1, gt2)


def test_push_and_transposed_forms_agree(c4):
    g = c4["g"]
    gp1, gt1 = _grads(c4, True)
    saved, g.nl.col_t = g.nl.col_t, None       # the push form
    try:
        gp2, gt2 = _grads(c4, True)
    finally:
        g.nl.col_t = saved
    assert torch.equal(gt1, gt2)
    assert float((gp1 - gp2).abs().max()) <= 1e-13 * float(gp1.abs().max())


def test_phi_gradient_matches_central_difference(c4):
    gphi, _ = _grads(c4, True)
    n = c4["g"].n
    v = torch.as_tensor(np.random.default_rng(21).uniform(-1.0, 1.0, n), device=DEV)
    lp = _lap(c4, c4["phi"] + FD_STEP * v, c4["theta"])
    lm = _lap(c4, c4["phi"] - FD_STEP * v, c4["theta"])
    fd = _dloss(c4, lp, lm) / (2 * FD_STEP)
    ad = float((gphi * v).sum())
    print(f"\ndirectional d/dphi: adjoint {ad:.12e} central difference {fd:.12e} rel {abs(ad - fd) / abs(fd):.2e}")
    assert abs(ad - fd) <= FD_TOL * abs(fd)


def test_theta_gradient_matches_central_differences(c4):
    _, gth = _grads(c4, True)
    fd = np.zeros(16)
    for t in range(16):
        e = torch.zeros(16, dtype=torch.float64)
        e[t] = FD_STEP
        e = e.reshape(4, 4)
        lp = _lap(c4, c4["phi"], c4["theta"] + e)
        lm = _lap(c4, c4["phi"], c4["theta"] - e)
        fd[t] = _dloss(c4, lp, lm) / (2 * FD_STEP)
    ad = gth.reshape(-1).cpu().numpy()
    # per coefficient, relative to its own size with a floor of 1e-3 of the
    # largest (so that a small coefficient cannot hide behind a large one)
    scale = np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    rel = np.abs(ad - fd) / scale
    print(f"\nd/dtheta vs central differences, per coefficient: {np.array2string(rel, precision=1)}")
    assert rel.max() <= FD_TOL


def test_theta_gradient_matches_oracle_on_the_full_set(c4):
    """d/dtheta on all 2.1M particles against the oracle's complex-step
    sensitivity, fed with the oracle's own Laplacian (for u) and projected
    derivatives D^ (every row evaluated by the oracle), per coefficient."""
    w = c4["w"]
    _, gth = _grads(c4, True)
    csr = O.neighbors(w.pos, w.R)
    rec, fl = O.sph2(w.pos, w.vol, w.phi[0], w.kernel, w.R, w.mapspec, csr=csr)
    assert not fl.any()
    u = 2.0 * (rec[:, 0, O.I_LAP] - w.extra["target"])
    nt = w.mapspec.as_array().shape[0]
    ref = O.dtheta(w.pos, w.mapspec, u, rec[:, 0, O.I_DHAT], np.arange(nt - 16, nt))
    ad = gth.reshape(-1).cpu().numpy()
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    rel = np.abs(ad - ref) / scale
    print(f"\nd/dtheta vs the oracle on {w.n} particles, per coefficient: {np.array2string(rel, precision=1)}")
    assert rel.max() <= 1e-6


def test_phi_gradient_matches_oracle_at_sampled_particles(c4):
    w, g = c4["w"], c4["g"]
    gphi, _ = _grads(c4, True)
    gphi = g.unsort(gphi).cpu().numpy()
    rng = np.random.default_rng(22)
    ks = np.sort(rng.choice(w.n, 48, replace=False))
    csr = O.neighbors(w.pos, w.R)
    rp, col = csr
    need = np.unique(np.concatenate([ks] + [col[rp[k]:rp[k + 1]] for k in ks]))
    rec, fl = O.sph2(w.pos, w.vol, w.phi[0], w.kernel, w.R, w.mapspec, rows=need)
    assert not fl.any()
    u = np.zeros(w.n)
    u[need] = 2.0 * (rec[:, 0, O.I_LAP] - w.extra["target"][need])
    ref = O.adjoint_dphi(w.pos, w.vol, w.kernel, w.R, w.mapspec, u, ks=ks, csr=csr)
    err = np.abs(gphi[ks] - ref).max() / np.abs(ref).max()
    print(f"\nd/dphi vs FP64 oracle at 48 particles: {err:.2e}")
    assert err <= 1e-9


def test_memory_held_between_forward_and_backward():
    """Between forward and backward each recompute mode keeps only what its
    backward reads: the FP64 state (keep), the moment sums (solve), nothing
    (recompute); the geometry itself keeps neither."""
    from paper_2607_28872_amd.autograd import ADJ_MASK, VctLaplacian
    w = I.small("sigma3d-adj")
    ms = w.mapspec
    base = I.MapSpec(ms.kind, ms.Hhat, ms.H, ms.dmin, ms.eps, list(ms.terms[:-16]))
    theta = torch.tensor(w.extra["theta"].reshape(4, 4), dtype=torch.float64, requires_grad=True)
    n = w.n
    state_b = vct.vct_state_stride(3, ADJ_MASK) * n * 8
    sums_b = vct.lib().vct_moments_workspace_size(3, n)
    held, grads = {}, {}
    for mode in (True, "solve", False):
        g = vct.Geometry(w.pos, w.vol, w.lo, w.hi, w.R, w.kernel, device=DEV)
        phi = g.sorted_field(w.phi[0])[0].clone().requires_grad_(True)
        torch.cuda.synchronize()
        m0 = torch.cuda.memory_allocated()
        lap = VctLaplacian.apply(phi, theta, g, base, mode)
        torch.cuda.synchronize()
        held[mode] = torch.cuda.memory_allocated() - m0
        ctx = lap.grad_fn
        assert g.state64 is None or mode is False
        assert g.ws_mom is None
        kept_state = 0 if ctx.state is None else ctx.state.numel() * ctx.state.element_size()
        kept_ws = 0 if ctx.ws is None else ctx.ws.numel()
        assert (kept_state, kept_ws) == {True: (0, 0), "solve": (0, sums_b), False: (state_b, 0)}[mode]
        lap.sum().backward()
        grads[mode] = phi.grad.clone()
        del lap, ctx, g, phi
        torch.cuda.empty_cache()
    print(f"\nallocated between forward and backward: {held} (state {state_b} B, moment sums {sums_b} B)")
    assert held[True] < held["solve"] < held[False]
    assert torch.equal(grads[True], grads["solve"]) and torch.equal(grads[True], grads[False])
