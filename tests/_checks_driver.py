"""Child process of test_gpu_checks.py: one small evaluation of every kernel
family through the C ABI with the library that VCT_LIB names, saved with the
device-check state.

  python tests/_checks_driver.py OUT.npz valid   -> outputs of the valid set
  python tests/_checks_driver.py OUT.npz plant   -> one window offset set one
                                                    past its chunk's window,
                                                    then the FP64 apply
"""
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_2607_28872_amd import inputs as I  # noqa: E402
from paper_2607_28872_amd import vct  # noqa: E402

DEV = "cuda:0"
ALL = (vct.VCT_OUT_GRAD | vct.VCT_OUT_LAP | vct.VCT_OUT_CROSS | vct.VCT_OUT_HESS | vct.VCT_OUT_PGRAD
       | vct.VCT_OUT_PHESS)


def main(out, mode):
    print(f"checks driver: {mode}, library {os.environ.get('VCT_LIB', vct.LIB_PATH)}", flush=True)
    w = I.small("sigma3d")
    ms = w.mapspec
    g = vct.Geometry(w.pos, w.vol, w.lo, w.hi, w.R, w.kernel, device=DEV, keep_col=False)
    phi = g.sorted_field(w.phi)
    res = {"row_ptr": g.row_ptr.cpu().numpy(), "col16": g.col16[: g.nnz].cpu().numpy()}
    if mode == "plant":
        g.moments(ms, ALL)
        i = g.n // 2
        nch = int(g.chunk_off[-1].item())
        cstart = g.chunk_start[: nch + 1].cpu().numpy()
        b = int(np.searchsorted(cstart, i, side="right") - 1)
        win = g.chunk_win[b].cpu().numpy()
        W = int(win[20 + win[0]])   # the window's size: off[nr]
        e = int(res["row_ptr"][i])
        g.col16[e] = W
        torch.cuda.synchronize()
        res["planted"] = np.array([i, e, W])
        res["apply"] = g.apply(phi).cpu().numpy()
    else:
        g.moments(ms, ALL, fp32_copy=True)
        res["state"] = g.state64.cpu().numpy()
        res["apply64"] = g.apply(phi).cpu().numpy()
        res["apply32"] = g.apply(phi, vct.VCT_MIXED).cpu().numpy()
        res["apply0"] = g.apply0(ms, phi, ALL).cpu().numpy()
        g.moments(ms, vct.VCT_OUT_LAP | vct.VCT_OUT_PZ)
        proj = g.apply(phi[:1].contiguous())
        u = torch.as_tensor(np.random.default_rng(3).standard_normal(g.n), device=DEV)
        dphi, dth = g.adjoint(u, proj)
        res["dphi"], res["dtheta"] = dphi.cpu().numpy(), dth.cpu().numpy()
        mask = vct.VCT_OUT_LAP | vct.VCT_OUT_PGRAD | vct.VCT_OUT_PHESS
        g.moments(ms, mask)
        proj = g.apply(phi[:1].contiguous())
        dth2, dz = g.adjoint_r2(phi[0].contiguous(), u, proj, want_dzhat=True)
        res["r2_dtheta"], res["r2_dz"] = dth2.cpu().numpy(), dz.cpu().numpy()
        J = g.map_alpha(ms)
        jb = J * torch.as_tensor(I.volume_perturbation(g.n), device=DEV)
        res["jbar"] = g.jbar_smooth(J, jb, 1e-2).cpu().numpy()
        # the neighbour search with windows over several LDS segments (hit
        # words, then their expansion) and with windows wider than the hit
        # words hold (the fill pass)
        for name, Rs in (("multiseg", 1.3), ("fill", 1.6)):
            gw = vct.Geometry(w.pos, w.vol, w.lo, w.hi, Rs * w.R, w.kernel, device=DEV, keep_col=False)
            res[f"row_ptr_{name}"] = gw.row_ptr.cpu().numpy()
            res[f"col16_{name}"] = gw.col16[: gw.nnz].cpu().numpy()
    checked, bits = vct.vct_device_checks()
    res["checked"], res["bits"] = np.array(int(checked)), np.array(bits)
    np.savez(out, **res)
    print(f"checks driver: done, checked={checked} bits={bits}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1], sys.argv[2])
