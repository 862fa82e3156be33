"""torch.autograd bridge for the physical Laplacian and its hand-written adjoint.

`VctLaplacian.apply(phi, theta, geom, base_map, recompute)` returns the
physical Laplacian (paper Sec. 2.1, Eq. lap_VCT, with the SPH(2) operators of
Sec. 3.1) of the field `phi` (sorted order, FP64, on the geometry's device)
under the vertical transformation `base_map` whose bottom elevation is
perturbed by sum_{m,n<4} theta[m, n] c_m(x) c_n(y), with
c in {1, cos 2 pi s, sin 2 pi s, cos 4 pi s}.  Its backward calls the adjoint
kernels (vct_apply_ops_adjoint) for d/dphi and d/dtheta; projected positions
are held fixed, so theta enters only through the mapping coefficients.

Between forward and backward the function holds, per particle:
  recompute=False    the FP64 state of the adjoint's rows (66 values in 3-D);
  recompute="solve"  the moment sums only (41 values in 3-D); the backward
                     runs the solve alone (vct_moments_resolve);
  recompute=True     neither; the backward runs vct_moments again.
Each mode runs the same kernels on the same inputs, so all three give the
same bits.  The forward releases the geometry's own references to the state
and to the moment workspace, so that only what the mode keeps stays alive.

`VctLaplacianR2.apply(phi, theta, phys, vol, box, base_map)` is the same
Laplacian with the particles' PHYSICAL positions held fixed: the forward
projects them with the perturbed mapping (z^ = alpha (z + beta)), builds the
geometry there and applies the operator; phi and the result are in the
caller's particle order.  Its backward gives d/dphi (the same adjoint as
above) and d/dtheta through the moving projected heights
(vct_apply_ops_adjoint_r2).
"""
from __future__ import annotations

import numpy as np
import torch

from . import vct

# the Laplacian and the projected derivatives its mapping coefficients multiply
ADJ_MASK = vct.VCT_OUT_LAP | vct.VCT_OUT_PZ

# perturbation basis of the bathymetry: (basis kind, frequency)
_B_ONE, _B_COS, _B_SIN = 0, 2, 3
PERTURBATION_BASIS = [(_B_ONE, 0.0), (_B_COS, 1.0), (_B_SIN, 1.0), (_B_COS, 2.0)]


def perturbation_terms(theta):
    """16 bottom terms theta[m, n] c_m(x) c_n(y) as (coef, bx, fx, by, fy)."""
    th = np.asarray(theta, dtype=np.float64).reshape(4, 4)
    return [(float(th[m, k]), bx, fx, by, fy)
            for m, (bx, fx) in enumerate(PERTURBATION_BASIS)
            for k, (by, fy) in enumerate(PERTURBATION_BASIS)]


class VctLaplacian(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, theta, geom, base_map, recompute=True):
        spec = base_map.with_terms(perturbation_terms(theta.detach().cpu().numpy()))
        st = geom.moments(spec, ADJ_MASK)
        if st < 0:
            raise vct.VctError("vct_moments", st)
        # one FP64 apply gives the Laplacian (row 0) and the projected
        # derivatives the bathymetry adjoint needs (the remaining rows)
        proj = geom.apply(phi.reshape(1, -1).contiguous(), vct.VCT_FP64)
        lap = proj[0, : geom.n, 0].clone()
        ctx.proj = proj
        ctx.geom, ctx.spec, ctx.recompute = geom, spec, recompute
        ctx.nbase = len(base_map.terms)
        ctx.theta_meta = (theta.dtype, theta.device)
        solve_only = isinstance(recompute, str) and recompute == "solve"
        ctx.state = None if recompute else geom.state64
        ctx.ws = geom.ws_mom if solve_only else None
        geom.ws_mom = None
        if recompute:
            geom.state64 = None
        ctx.save_for_backward(phi)
        return lap

    @staticmethod
    def backward(ctx, grad_lap):
        (phi,) = ctx.saved_tensors
        g = ctx.geom
        if isinstance(ctx.recompute, str) and ctx.recompute == "solve":
            st = g.resolve(ctx.spec, ADJ_MASK, ws=ctx.ws)
            if st < 0:
                raise vct.VctError("vct_moments_resolve", st)
        elif ctx.recompute:
            st = g.moments(ctx.spec, ADJ_MASK)
            if st < 0:
                raise vct.VctError("vct_moments", st)
        else:
            g.state64, g.mask, g.cmap = ctx.state, ADJ_MASK, vct.make_map(ctx.spec)
        u = grad_lap.to(torch.float64).contiguous()
        dphi, dth = g.adjoint(u, ctx.proj, want_dtheta=ctx.needs_input_grad[1])
        dtheta = None
        if dth is not None:
            dtype, dev = ctx.theta_meta
            dtheta = dth[ctx.nbase:].to(device=dev, dtype=dtype).reshape(4, 4)
        return dphi.reshape(phi.shape), dtheta, None, None, None


def laplacian_loss(geom, phi, theta, base_map, target, recompute=True):
    """sum_i (lap_i - target_i)^2 on sorted particles, differentiable in phi and theta."""
    lap = VctLaplacian.apply(phi, theta, geom, base_map, recompute)
    return ((lap - target) ** 2).sum()


# the Laplacian and the projected derivatives the position adjoint reads
R2_MASK = vct.VCT_OUT_LAP | vct.VCT_OUT_PGRAD | vct.VCT_OUT_PHESS


class VctLaplacianR2(torch.autograd.Function):
    """phi: (n,) FP64 in the caller's order; theta: (4, 4); phys: (dim, n)
    physical positions (device tensor); vol: (n,); box: (lo, hi, R, kernel)."""

    @staticmethod
    def forward(ctx, phi, theta, phys, vol, box, base_map):
        lo, hi, R, kernel = box
        spec = base_map.with_terms(perturbation_terms(theta.detach().cpu().numpy()))
        cmap = vct.make_map(spec)
        phys = phys.to(torch.float64).contiguous()
        pos = torch.empty_like(phys)
        vct.vct_map_project(phys.shape[0], phys.shape[1], phys, cmap, pos)
        geom = vct.Geometry(pos, vol, lo, hi, R, kernel, device=phys.device, keep_col=False)
        st = geom.moments(spec, R2_MASK)
        if st < 0:
            raise vct.VctError("vct_moments", st)
        phis = geom.sorted_field(phi.detach())
        proj = geom.apply(phis, vct.VCT_FP64)
        ctx.geom, ctx.proj, ctx.phis = geom, proj, phis
        ctx.nbase = len(base_map.terms)
        ctx.theta_meta = (theta.dtype, theta.device)
        return geom.unsort(proj[0, : geom.n, 0].contiguous())

    @staticmethod
    def backward(ctx, grad_lap):
        g = ctx.geom
        u = g.sorted_field(grad_lap.to(torch.float64))[0].contiguous()
        dphi = None
        if ctx.needs_input_grad[0]:
            dphi_s, _ = g.adjoint(u, ctx.proj, want_dtheta=False)
            dphi = g.unsort(dphi_s.contiguous())
        dtheta = None
        if ctx.needs_input_grad[1]:
            dth, _ = g.adjoint_r2(ctx.phis[0].contiguous(), u, ctx.proj)
            dtype, dev = ctx.theta_meta
            dtheta = dth[ctx.nbase:].to(device=dev, dtype=dtype).reshape(4, 4)
        return dphi, dtheta, None, None, None, None
