"""Helpers shared by the GPU parity tests: map library output rows to the
oracle's record slots and measure normwise errors."""
import numpy as np

import oracle as O
from paper_2607_28872_amd import vct

ALL_OUT = (vct.VCT_OUT_GRAD | vct.VCT_OUT_LAP | vct.VCT_OUT_CROSS | vct.VCT_OUT_HESS | vct.VCT_OUT_PGRAD
           | vct.VCT_OUT_PHESS)


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
        ]
    else:
        groups = [
            (vct.VCT_OUT_GRAD, [0, 2], [1, 1]),
            (vct.VCT_OUT_LAP, [3], [1]),
            (vct.VCT_OUT_CROSS, [5], [1]),
            (vct.VCT_OUT_HESS, [7, 9, 11], [1, 1, 1]),
            (vct.VCT_OUT_PGRAD, [13, 15] if g1 else [16, 18], [1, 1]),
            (vct.VCT_OUT_PHESS, [19, 21, 23], [1, 1, 0.5]),
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
                 (vct.VCT_OUT_PHESS, ["pxx", "pyy", "pzz", "pxy", "pxz", "pyz"])]
    else:
        table = [(vct.VCT_OUT_GRAD, ["gx", "gz"]), (vct.VCT_OUT_LAP, ["lap"]), (vct.VCT_OUT_CROSS, ["xz"]),
                 (vct.VCT_OUT_HESS, ["Hxx", "Hzz", "Hxz"]), (vct.VCT_OUT_PGRAD, ["pgx", "pgz"]),
                 (vct.VCT_OUT_PHESS, ["pxx", "pzz", "pxz"])]
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
