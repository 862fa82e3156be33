"""SPH(2) operators of selected particles evaluated in x87 extended precision.

Test infrastructure, like the rest of this package: only the tests, the smoke
check and the CPU baseline of the benchmark use it.

The FP64 oracle (orc_sph2) solves the paper's moment system (Sec. 3.1,
Eqs. gra_1st and sec_SPH2) exactly as written, and on anisotropic or
ellipsoidal neighbourhoods the rounding of its FP64 sums is amplified by the
conditioning of M_i to a few 1e-12 (relative to the largest value of a row).
This module takes the same steps in the same order with numpy's long double
(64-bit significand on x86-64), so its own rounding is about 2000 times
smaller; it is the reference that separates the FP64 oracle's rounding from
that of the implementation under test.  It is slow (Python loops over the
neighbours) and meant for a few hundred particles.

Steps for particle i with neighbours j (r_ij = x_j - x_i, V_j the volume):
  grad w_ij = -(dw/dr) r_ij / |r_ij|          (kernel of Sec. 4 / Wendland C2)
  A_i = sum_j V_j grad w_ij r_ij^T,  L_i = A_i^-1           (Eq. gra_1st)
  g1_i = sum_j V_j phi_ij L_i grad w_ij
  q_ij = second-order monomials of r_ij,  Q_i = sum_j V_j q_ij (L_i grad w_ij)^T
  F_ij = r_ij . (L_i grad w_ij) / |r_ij|^4,  p_ij = q_ij - Q_i r_ij
  M_i = sum_j V_j F_ij q_ij p_ij^T                          (Eq. sec_SPH2)
  b_i = sum_j V_j F_ij q_ij (phi_ij - r_ij . g1_i),  D_i = 2 M_i^-1 b_i
  g2_i = g1_i - Q_i^T D_i / 2
and then the transformed-coordinate outputs of Sec. 2.1 (Eqs. grad_VCT,
lap_VCT) with the FP64 map coefficients of the C oracle (orc_map_eval).
Records use the C oracle's layout (REC slots).
"""
import numpy as np

from . import REC, map_eval, neighbors

LD = np.longdouble
_PI = LD("3.14159265358979323846264338327950288")


def available():
    """True when long double carries more precision than double."""
    return np.finfo(LD).eps < 1e-18


def _kernel(kernel, dim, R, r):
    """w and dw/dr (Wendland C2 for kernel 0, cubic spline with l = R/2 for 1)."""
    if kernel == 0:
        C = LD(7) / (_PI * R * R) if dim == 2 else LD(21) / (2 * _PI * R * R * R)
        q = r / R
        if q >= 1:
            return LD(0), LD(0)
        a = 1 - q
        return C * a ** 4 * (1 + 4 * q), C * (-20 * q * a ** 3) / R
    l = R / 2
    ad = LD(10) / (7 * _PI * l * l) if dim == 2 else LD(1) / (_PI * l ** 3)
    s = r / l
    if s <= 1:
        return ad * (1 - LD(1.5) * s * s + LD(0.75) * s ** 3), ad * (-3 * s + LD(2.25) * s * s) / l
    if s < 2:
        t = 2 - s
        return ad * LD(0.25) * t ** 3, ad * (LD(-0.75) * t * t) / l
    return LD(0), LD(0)


def _solve(A, B):
    """Gaussian elimination with partial pivoting in long double."""
    A = A.copy()
    B = B.copy()
    n = A.shape[0]
    for c in range(n):
        p = c + int(np.argmax(np.abs(A[c:, c])))
        if p != c:
            A[[c, p]] = A[[p, c]]
            B[[c, p]] = B[[p, c]]
        for r in range(c + 1, n):
            f = A[r, c] / A[c, c]
            A[r, c:] -= f * A[c, c:]
            B[r] -= f * B[c]
    X = np.zeros_like(B)
    for c in range(n - 1, -1, -1):
        X[c] = (B[c] - A[c, c + 1:] @ X[c + 1:]) / A[c, c]
    return X


def _monomials(dim, r):
    if dim == 2:
        return np.array([r[0] * r[0], r[1] * r[1], r[0] * r[1]], dtype=LD)
    return np.array([r[0] * r[0], r[1] * r[1], r[2] * r[2], r[0] * r[1], r[0] * r[2], r[1] * r[2]], dtype=LD)


def _particle(dim, pos, vol, phis, kernel, R, i, nb, grad_order):
    """(nf, 2 d + ...) computational results of one particle: g1, g2, D."""
    rs, gws, qs, Vs = [], [], [], []
    for j in nb:
        r = pos[:, j] - pos[:, i]
        rr = np.sqrt(np.sum(r * r))
        _, dw = _kernel(kernel, dim, R, rr)
        rs.append(r)
        gws.append(-dw * r / rr)
        qs.append(_monomials(dim, r))
        Vs.append(vol[j])
    rs, gws, qs, Vs = np.array(rs), np.array(gws), np.array(qs), np.array(Vs)
    A = np.einsum("k,ka,kb->ab", Vs, gws, rs)
    L = _solve(A, np.eye(dim, dtype=LD))
    gt = gws @ L.T
    Q = np.einsum("k,km,ka->ma", Vs, qs, gt)
    d2 = np.sum(rs * rs, axis=1)
    F = np.sum(rs * gt, axis=1) / (d2 * d2)
    p = qs - rs @ Q.T
    M = np.einsum("k,km,kn->mn", Vs * F, qs, p)
    cond = float(np.linalg.cond(M.astype(np.float64)))
    res = []
    for ph in phis:
        phij = ph[nb] - ph[i]
        g1 = np.einsum("k,k,ka->a", Vs, phij, gt)
        b = np.einsum("k,k,km->m", Vs * F, phij - rs @ g1, qs)
        D = 2 * _solve(M, b.reshape(-1, 1)).ravel()
        g2 = g1 - LD(0.5) * (Q.T @ D)
        res.append((g1, g2, D, g1 if grad_order == 1 else g2))
    return res, cond


def sph2_extended(pos, vol, phi, kernel, R, mapspec, rows, grad_order=2, with_cond=False):
    """Records (len(rows), nf, REC) as float64, computed in long double.  phi
    may be given in long double (exact test fields); pos and vol are FP64.
    With with_cond, also the 2-norm condition number of every M_i."""
    pos64 = np.ascontiguousarray(pos, dtype=np.float64)
    dim, n = pos64.shape
    posl = pos64.astype(LD)
    voll = np.asarray(vol, dtype=np.float64).astype(LD)
    phil = np.atleast_2d(np.asarray(phi)).astype(LD)   # long double input kept as is
    rows = np.asarray(rows, dtype=np.int64)
    rp, col = neighbors(pos64, R, rows=rows)
    x = pos64[0, rows]
    y = pos64[1, rows] if dim == 3 else None
    zh = pos64[dim - 1, rows]
    mc = map_eval(dim, x, y, zh, mapspec).astype(LD)
    out = np.zeros((rows.shape[0], phil.shape[0], REC))
    conds = np.zeros(rows.shape[0])
    for k, i in enumerate(rows):
        nb = col[rp[k]:rp[k + 1]]
        Jm = mc[k, 0:9].reshape(3, 3)
        ct = mc[k, 9:15]
        hz = mc[k, 15:24].reshape(3, 3)
        res, conds[k] = _particle(dim, posl, voll, phil, kernel, LD(R), i, nb, grad_order)
        for f, (g1, g2, D, gs) in enumerate(res):
            gh = np.zeros(3, dtype=LD)
            Hh = np.zeros((3, 3), dtype=LD)
            g1e = np.zeros(3, dtype=LD)
            g2e = np.zeros(3, dtype=LD)
            De = np.zeros(6, dtype=LD)
            if dim == 2:
                gh[0], gh[2] = gs[0], gs[1]
                g1e[0], g1e[2] = g1[0], g1[1]
                g2e[0], g2e[2] = g2[0], g2[1]
                Hh[0, 0], Hh[2, 2] = D[0], D[1]
                Hh[0, 2] = Hh[2, 0] = LD(0.5) * D[2]
                De[0], De[2], De[4] = D[0], D[1], D[2]
            else:
                gh[:], g1e[:], g2e[:] = gs, g1, g2
                Hh[0, 0], Hh[1, 1], Hh[2, 2] = D[0], D[1], D[2]
                Hh[0, 1] = Hh[1, 0] = LD(0.5) * D[3]
                Hh[0, 2] = Hh[2, 0] = LD(0.5) * D[4]
                Hh[1, 2] = Hh[2, 1] = LD(0.5) * D[5]
                De[:] = D
            Dhat = np.array([gh[2], Hh[0, 0], Hh[1, 1], Hh[2, 2], Hh[0, 2], Hh[1, 2]], dtype=LD)
            lap = np.sum(ct * Dhat)
            gp = Jm @ gh
            Hp = Jm @ Hh @ Jm.T + gh[2] * hz
            if dim == 2:
                gp[1] = 0
                Hp[1, :] = 0
                Hp[:, 1] = 0
            rec = out[k, f]
            rec[0:3] = gp.astype(np.float64)
            rec[3] = float(lap)
            rec[4:7] = [float(Hp[0, 1]), float(Hp[0, 2]), float(Hp[1, 2])]
            rec[7:13] = [float(Hp[0, 0]), float(Hp[1, 1]), float(Hp[2, 2]),
                         float(Hp[0, 1]), float(Hp[0, 2]), float(Hp[1, 2])]
            rec[13:16] = g1e.astype(np.float64)
            rec[16:19] = g2e.astype(np.float64)
            rec[19:25] = De.astype(np.float64)
            rec[25:31] = Dhat.astype(np.float64)
            rec[31] = float(Hp[0, 0] + Hp[1, 1] + Hp[2, 2])
    return (out, conds) if with_cond else out


def moment_condition(pos, vol, kernel, R, rows=None, block=200000):
    """2-norm condition number of M_i for the given particles (all if rows is
    None): FP64, vectorised over the neighbour pairs in blocks of rows; a
    diagnostic for error bounds, not an operator."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    vol = np.asarray(vol, dtype=np.float64)
    dim, n = pos.shape
    rows = np.arange(n) if rows is None else np.asarray(rows, dtype=np.int64)
    out = np.empty(rows.shape[0])
    for b0 in range(0, rows.shape[0], block):
        rb = rows[b0:b0 + block]
        rp, col = neighbors(pos, R, rows=rb)
        out[b0:b0 + block] = _cond_block(pos, vol, kernel, R, rb, rp, col)
    return out


def _cond_block(pos, vol, kernel, R, rb, rp, col):
    dim = pos.shape[0]
    owner = np.repeat(np.arange(rb.shape[0]), np.diff(rp))
    r = (pos[:, col] - pos[:, rb[owner]]).T                     # (nnz, d)
    rr = np.sqrt(np.sum(r * r, axis=1))
    dw = _dwdr64(kernel, dim, R, rr)
    gw = -(dw / rr)[:, None] * r
    V = vol[col]

    def seg(x):
        return np.add.reduceat(x, rp[:-1], axis=0)

    A = seg(V[:, None, None] * gw[:, :, None] * r[:, None, :])
    L = np.linalg.inv(A)
    gt = np.einsum("kab,kb->ka", L[owner], gw)
    if dim == 2:
        q = np.stack([r[:, 0] ** 2, r[:, 1] ** 2, r[:, 0] * r[:, 1]], axis=1)
    else:
        q = np.stack([r[:, 0] ** 2, r[:, 1] ** 2, r[:, 2] ** 2, r[:, 0] * r[:, 1], r[:, 0] * r[:, 2],
                      r[:, 1] * r[:, 2]], axis=1)
    Q = seg(V[:, None, None] * q[:, :, None] * gt[:, None, :])
    F = np.sum(r * gt, axis=1) / rr ** 4
    p = q - np.einsum("kma,ka->km", Q[owner], r)
    M = seg((V * F)[:, None, None] * q[:, :, None] * p[:, None, :])
    return np.linalg.cond(M)


def _dwdr64(kernel, dim, R, r):
    """dw/dr in FP64, vectorised (same formulas as _kernel)."""
    if kernel == 0:
        C = 7.0 / (np.pi * R * R) if dim == 2 else 21.0 / (2 * np.pi * R ** 3)
        q = r / R
        return np.where(q < 1.0, C * (-20.0 * q * (1.0 - q) ** 3) / R, 0.0)
    l = 0.5 * R
    ad = 10.0 / (7 * np.pi * l * l) if dim == 2 else 1.0 / (np.pi * l ** 3)
    s = r / l
    inner = ad * (-3.0 * s + 2.25 * s * s) / l
    outer = ad * (-0.75 * (2.0 - s) ** 2) / l
    return np.where(s <= 1.0, inner, np.where(s < 2.0, outer, 0.0))
