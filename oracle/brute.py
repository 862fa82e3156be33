"""Independent numpy cross-checks for the C oracle (test infrastructure only).

* brute_neighbors: O(N^2) neighbour lists by the literal set definition
  S_i = { j != i : |r_ij| < r_e } (paper Eq. SPH_neighbor_set), with the
  squared distance summed left to right in FP64 as in the C oracle.
* block_solve: the SPH(2) estimate written as one (d+m) x (d+m) linear system.
  Expanding phi_ij = r_ij . grad phi + 1/2 q_ij . D phi (D carries twice the
  mixed second derivatives) and taking moments against V_j grad w_ij (d rows)
  and V_j F_ij q_ij (m rows) gives
      [ A  B ] [ grad phi ]   [ a ]      A = sum V grad w r^T,  B = sum V grad w q^T
      [ C  E ] [ D phi / 2] = [ s ],     C = sum V F q r^T,     E = sum V F q q^T
  with a = sum V phi_ij grad w and s = sum V F q phi_ij.  Eliminating the first
  block row with L = A^-1 reproduces the two-stage form of paper Eq. sec_SPH2,
  so this dense solve is an independent route to the same D and to the
  second-order gradient (paper Sec. 3.1 notes that SPH(2) also yields one).
"""
from __future__ import annotations

import numpy as np


def brute_neighbors(pos, R):
    pos = np.asarray(pos, dtype=np.float64)
    dim, n = pos.shape
    R2 = R * R
    rows = []
    for i in range(n):
        d2 = (pos[0] - pos[0, i]) * (pos[0] - pos[0, i])
        d2 = d2 + (pos[1] - pos[1, i]) * (pos[1] - pos[1, i])
        if dim == 3:
            d2 = d2 + (pos[2] - pos[2, i]) * (pos[2] - pos[2, i])
        m = d2 < R2
        m[i] = False
        rows.append(np.nonzero(m)[0].astype(np.int32))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([len(r) for r in rows])
    col = np.concatenate(rows) if rows else np.zeros(0, np.int32)
    return row_ptr, col


def wendland_grad_factor(r, R, dim):
    """grad_i w(|r_ij|) = factor * r_ij for Wendland C2 (textbook normalisation)."""
    C = 7.0 / (np.pi * R * R) if dim == 2 else 21.0 / (2.0 * np.pi * R ** 3)
    q = r / R
    return np.where(q < 1.0, C * 20.0 * (1.0 - q) ** 3 / (R * R), 0.0)


def monomials(r):
    """q for difference vectors r (dim, k): 2-D [x^2, z^2, xz], 3-D [x^2, y^2, z^2, xy, xz, yz]."""
    if r.shape[0] == 2:
        return np.stack([r[0] * r[0], r[1] * r[1], r[0] * r[1]])
    return np.stack([r[0] * r[0], r[1] * r[1], r[2] * r[2], r[0] * r[1], r[0] * r[2], r[1] * r[2]])


def block_solve(pos, vol, phi, R, i, nb):
    """Dense-system SPH(2) at particle i (Wendland kernel): returns
    (grad2 (d,), D (m,)) in the projected space."""
    pos = np.asarray(pos, dtype=np.float64)
    dim = pos.shape[0]
    r = pos[:, nb] - pos[:, i:i + 1]
    rr = np.sqrt((r * r).sum(0))
    gw = wendland_grad_factor(rr, R, dim) * r
    V = vol[nb]
    q = monomials(r)
    A = (V * gw) @ r.T
    L = np.linalg.inv(A)
    gt = L @ gw
    F = (r * gt).sum(0) / rr ** 4
    B = (V * gw) @ q.T
    Cm = (V * F * q) @ r.T
    E = (V * F * q) @ q.T
    K = np.block([[A, B], [Cm, E]])
    phij = phi[nb] - phi[i]
    rhs = np.concatenate([(V * phij * gw).sum(1), (V * F * phij * q).sum(1)])
    sol = np.linalg.solve(K, rhs)
    return sol[:dim], 2.0 * sol[dim:]
