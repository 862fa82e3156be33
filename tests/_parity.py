"""Helpers shared by the GPU parity tests: map library output rows to the
oracle's record slots and measure normwise errors."""
import numpy as np

import oracle as O
from oracle import extended as OX
from paper_2607_28872_amd import vct

FP64_TOL = 1e-12
FP64_ORACLE_TOL = 1e-11
EXT_KAPPA = 1e-13        # GPU vs extended precision, per unit of kappa_i
ORC_KAPPA = 1e-11        # GPU vs FP64 oracle (the oracle's own rounding dominates)

ALL_OUT = (vct.VCT_OUT_GRAD | vct.VCT_OUT_LAP | vct.VCT_OUT_CROSS | vct.VCT_OUT_HESS | vct.VCT_OUT_PGRAD
           | vct.VCT_OUT_PHESS | vct.VCT_OUT_PZ)


def oracle_rows(rec, dim, mask):
    """(n, nf, REC) oracle records -> (nf, n, n_out) in the library's row order."""
    cols, scale = [], []
    g1 = bool(mask & vct.VCT_OPT_GRAD1)
    if dim == 3:
        groups = [
            (vct.VCT_OUT_GRAD, [0, 1, 2], [1, 1, 1]),
            (vct.VCT_OUT_LAP, [3], [1]),
            (vct.VCT_OUT_CROSS, [4, 5, 6], [1, 1, 1]),
            (vct.VCT_OUT_HESS, [7, 8, 9, 10, 11, 12], [1] * 6),
            (vct.VCT_OUT_PGRAD, [13, 14, 15] if g1 else [16, 17, 18], [1, 1, 1]),
            (vct.VCT_OUT_PHESS, [19, 20, 21, 22, 23, 24], [1, 1, 1, 0.5, 0.5, 0.5]),
            (vct.VCT_OUT_PZ, [15 if g1 else 18, 21, 23, 24], [1, 1, 0.5, 0.5]),
        ]
    else:
        groups = [
            (vct.VCT_OUT_GRAD, [0, 2], [1, 1]),
            (vct.VCT_OUT_LAP, [3], [1]),
            (vct.VCT_OUT_CROSS, [5], [1]),
            (vct.VCT_OUT_HESS, [7, 9, 11], [1, 1, 1]),
            (vct.VCT_OUT_PGRAD, [13, 15] if g1 else [16, 18], [1, 1]),
            (vct.VCT_OUT_PHESS, [19, 21, 23], [1, 1, 0.5]),
            (vct.VCT_OUT_PZ, [15 if g1 else 18, 21, 23], [1, 1, 0.5]),
        ]
    for bit, c, s in groups:
        if mask & bit:
            cols += c
            scale += s
    out = rec[:, :, cols] * np.asarray(scale)[None, None, :]
    return np.transpose(out, (1, 0, 2))


def row_names(dim, mask):
    names = []
    if dim == 3:
        table = [(vct.VCT_OUT_GRAD, ["gx", "gy", "gz"]), (vct.VCT_OUT_LAP, ["lap"]),
                 (vct.VCT_OUT_CROSS, ["xy", "xz", "yz"]),
                 (vct.VCT_OUT_HESS, ["Hxx", "Hyy", "Hzz", "Hxy", "Hxz", "Hyz"]),
                 (vct.VCT_OUT_PGRAD, ["pgx", "pgy", "pgz"]),
                 (vct.VCT_OUT_PHESS, ["pxx", "pyy", "pzz", "pxy", "pxz", "pyz"]),
                 (vct.VCT_OUT_PZ, ["zgz", "zzz", "zxz", "zyz"])]
    else:
        table = [(vct.VCT_OUT_GRAD, ["gx", "gz"]), (vct.VCT_OUT_LAP, ["lap"]), (vct.VCT_OUT_CROSS, ["xz"]),
                 (vct.VCT_OUT_HESS, ["Hxx", "Hzz", "Hxz"]), (vct.VCT_OUT_PGRAD, ["pgx", "pgz"]),
                 (vct.VCT_OUT_PHESS, ["pxx", "pzz", "pxz"]), (vct.VCT_OUT_PZ, ["zgz", "zzz", "zxz"])]
    for bit, nm in table:
        if mask & bit:
            names += nm
    return names


def normwise(got, ref):
    """max |got - ref| / max |ref| per (field, row); rows with a zero reference
    use the absolute error."""
    err = np.abs(got - ref).max(axis=1)
    sc = np.abs(ref).max(axis=1)
    return np.where(sc > 0, err / np.where(sc > 0, sc, 1.0), err)


def per_particle(got, ref, scale):
    """max over fields and rows of |got - ref| / (largest |value| of the row)."""
    return (np.abs(got - ref) / scale).max(axis=(0, 2))


def fp64_check(w, kernel, R, got, ref, mask, grad_order=2, worst=48, extra=16, idx=None, scale=None, label=None):
    """Asserts the FP64 bar (see the GPU parity tests); got and ref are
    (nf, m, rows) for the particles idx (all if None).

    The bar is 1e-12 normwise (error over the largest reference value of the
    row) against the extended-precision evaluation, on the particles where the
    GPU and the FP64 oracle differ most plus a random sample.  A particle above
    1e-12 is an exception that must stay within EXT_KAPPA * kappa_i (kappa_i the
    condition number of its moment matrix); exceptions are listed in the
    output.  Against the FP64 oracle, whose own rounding reaches 5e-12 kappa_i,
    every particle must be within max(FP64_ORACLE_TOL, ORC_KAPPA * kappa_i).
    Prints the maxima against 1e-12 and returns (GPU vs oracle, GPU vs
    extended, oracle vs extended)."""
    idx = np.arange(w.n) if idx is None else np.asarray(idx)
    label = label or getattr(w, "name", "set")
    if scale is None:
        scale = np.abs(ref).max(axis=1, keepdims=True)
        scale = np.where(scale > 0, scale, 1.0)
    e_orc_all = per_particle(got, ref, scale)
    loose = np.nonzero(e_orc_all > FP64_ORACLE_TOL)[0]
    if loose.size:
        kap = OX.moment_condition(w.pos, w.vol, kernel, R, rows=idx[loose])
        bad = e_orc_all[loose] > ORC_KAPPA * kap
        assert not bad.any(), f"GPU vs FP64 oracle: {e_orc_all[loose][bad].max():.2e} at kappa {kap[bad].min():.2e}"
    if not OX.available():
        print(f"[FP64 bar 1e-12] {label}: GPU vs FP64 oracle {e_orc_all.max():.2e} on {idx.shape[0]} particles "
              "(no extended precision on this host)")
        return e_orc_all.max(), None, None
    rng = np.random.default_rng(11)
    sel = np.unique(np.concatenate([np.argsort(e_orc_all)[-worst:],
                                    rng.choice(idx.shape[0], min(extra, idx.shape[0]), replace=False)]))
    rows = idx[sel]
    ext = oracle_rows(OX.sph2_extended(w.pos, w.vol, w.phi, kernel, R, w.mapspec, rows, grad_order), w.dim, mask)
    kap = OX.moment_condition(w.pos, w.vol, kernel, R, rows=rows)
    e_gpu = per_particle(got[:, sel], ext, scale)
    e_ref = per_particle(ref[:, sel], ext, scale)
    over = np.nonzero(e_gpu > FP64_TOL)[0]
    print(f"\n[FP64 bar 1e-12] {label}: GPU vs extended precision {e_gpu.max():.2e} on {sel.shape[0]} particles "
          f"({'within' if over.size == 0 else 'ABOVE'} 1e-12); FP64 oracle vs extended {e_ref.max():.2e}; "
          f"GPU vs FP64 oracle {e_orc_all.max():.2e} on {idx.shape[0]} particles")
    if over.size:
        # the same extended-precision evaluation with every input (positions
        # and field values) moved by one ulp in a seeded random direction: the
        # change is what the FP64 representation of the inputs alone leaves
        # undetermined, a floor below which no FP64 evaluation can be held
        sens = input_ulp_sensitivity(w, kernel, R, rows[over], mask, grad_order, ext[:, over], scale)
        print(f"  kappa-scaled exceptions (particle, kappa, error, one-ulp input sensitivity): "
              + ", ".join(f"({int(rows[k])}, {kap[k]:.1f}, {e_gpu[k]:.2e}, {sens[m]:.1e})"
                          for m, k in enumerate(over)))
    assert np.all(e_gpu <= np.maximum(FP64_TOL, EXT_KAPPA * kap)), \
        f"GPU vs extended: worst {e_gpu.max():.2e} at kappa {kap[np.argmax(e_gpu)]:.2e}"
    return e_orc_all.max(), e_gpu.max(), e_ref.max()


def input_ulp_sensitivity(w, kernel, R, rows, mask, grad_order, ext, scale, seed=12):
    """Per particle (rows): the normwise change of the extended-precision
    outputs when every position and field value of the set is moved by one
    ulp up or down (seeded random signs)."""
    rng = np.random.default_rng(seed)
    pos = w.pos * (1.0 + np.finfo(np.float64).eps * rng.choice([-1.0, 1.0], size=w.pos.shape))
    phi = w.phi * (1.0 + np.finfo(np.float64).eps * rng.choice([-1.0, 1.0], size=w.phi.shape))
    pert = oracle_rows(OX.sph2_extended(pos, w.vol, phi, kernel, R, w.mapspec, rows, grad_order), w.dim, mask)
    return per_particle(pert, ext, scale)
