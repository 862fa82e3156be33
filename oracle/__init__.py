"""CPU FP64 oracle for the VCT-SPH(2) operators (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product path (the HIP library and its binding) never
imports, links or calls it, and the oracle never calls the product path.

The arithmetic lives in plain C (orc.c, FP64, OpenMP over particles); this
module only builds that file with gcc and marshals numpy arrays into it.
extended.py evaluates the same operators for selected particles in x87
extended precision, to separate the FP64 oracle's own rounding from that of
the code under test.
Record layout of sph2() outputs: see ORC_REC in orc.h (indices below).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")

# record indices (orc.h)
REC = 32
I_GRAD = slice(0, 3)
I_LAP = 3
I_CROSS = slice(4, 7)
I_HESS = slice(7, 13)
I_G1 = slice(13, 16)
I_G2 = slice(16, 19)
I_D = slice(19, 25)
I_DHAT = slice(25, 31)
I_LAP_TRACE = 31

F_FEW, F_SINGULAR_A, F_SINGULAR_M, F_NONFINITE, F_DUPLICATE, F_MAP = 1, 2, 4, 8, 16, 32


SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(verbose=False, sanitize=False, out=None):
    """Compile orc.c into liborc.so (plain gcc, no fused multiply-add).  With
    sanitize=True the same source is built with AddressSanitizer and
    UndefinedBehaviorSanitizer into `out` (for a run with the gcc ASan
    runtime preloaded; ORACLE_LIB names it to lib())."""
    src = os.path.join(HERE, "orc.c")
    dst = out or (os.path.join(HERE, "liborc_san.so") if sanitize else LIB_PATH)
    cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", *(SAN_FLAGS if sanitize else []), src, "-o", dst,
           "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    global _lib
    _lib = None
    return dst


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB") or LIB_PATH
        if not os.path.exists(path):
            build()
        L = C.CDLL(path)
        dp, ip64, ip32, u8p = (C.POINTER(C.c_double), C.POINTER(C.c_int64),
                               C.POINTER(C.c_int32), C.POINTER(C.c_uint8))
        L.orc_neighbors.restype = C.c_int64
        L.orc_neighbors.argtypes = [C.c_int, C.c_int64, dp, C.c_double, C.c_int64, ip64, C.c_int,
                                    ip64, ip32, C.c_int64]
        L.orc_sph2.restype = C.c_int
        L.orc_sph2.argtypes = [C.c_int, C.c_int64, dp, dp, C.c_int, dp, C.c_int, C.c_double,
                               C.c_int, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, dp,
                               C.c_int, C.c_int64, ip64, ip64, ip32, dp, u8p]
        L.orc_set_per_particle.restype = None
        L.orc_set_per_particle.argtypes = [dp, C.c_int64]
        L.orc_jbar_smooth.restype = C.c_int
        L.orc_jbar_smooth.argtypes = [C.c_int, C.c_int64, dp, dp, dp, C.c_double, C.c_double, ip64, ip64, ip32]
        L.orc_r2_dzhat.restype = C.c_int
        L.orc_r2_dzhat.argtypes = [C.c_int, C.c_int64, dp, dp, dp, C.c_int, C.c_double, C.c_int, C.c_double,
                                   C.c_double, C.c_double, C.c_double, C.c_int, dp, dp, C.c_int, C.c_int64, ip64,
                                   ip64, ip32, dp]
        L.orc_project.restype = C.c_int
        L.orc_project.argtypes = [C.c_int, C.c_int64, dp, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.c_int, dp, dp]
        L.orc_r2_dtheta.restype = C.c_int
        L.orc_r2_dtheta.argtypes = [C.c_int, C.c_int64, dp, dp, dp, dp, C.c_int, C.c_double, C.c_int, C.c_double,
                                    C.c_double, C.c_double, C.c_double, C.c_int, dp, C.c_int, ip32, ip64, ip32, dp]
        L.orc_adjoint_dphi.restype = C.c_int
        L.orc_adjoint_dphi.argtypes = [C.c_int, C.c_int64, dp, dp, C.c_int, C.c_double, C.c_int,
                                       C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, dp,
                                       C.c_int, ip64, ip32, dp, C.c_int64, ip64, dp]
        L.orc_dtheta.restype = C.c_int
        L.orc_dtheta.argtypes = [C.c_int, C.c_int64, dp, C.c_int, C.c_double, C.c_double, C.c_double,
                                 C.c_double, C.c_int, dp, dp, dp, C.c_int, ip32, dp]
        L.orc_map_eval.restype = C.c_int
        L.orc_map_eval.argtypes = [C.c_int, C.c_int64, dp, dp, dp, C.c_int, C.c_double, C.c_double,
                                   C.c_double, C.c_double, C.c_int, dp, C.c_int, dp]
        L.orc_alpha_beta.restype = C.c_int
        L.orc_alpha_beta.argtypes = [C.c_int, C.c_int64, dp, dp, C.c_int, C.c_double, C.c_double,
                                     C.c_double, C.c_double, C.c_int, dp, dp]
        L.orc_kernel_eval.restype = None
        L.orc_kernel_eval.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, dp, dp]
        L.orc_lap_weights.restype = C.c_int
        L.orc_lap_weights.argtypes = [C.c_int, C.c_int64, dp, dp, C.c_int, C.c_double, C.c_int, C.c_double,
                                      C.c_double, C.c_double, C.c_double, C.c_int, dp, C.c_int, C.c_int64, ip64,
                                      ip64, ip32, dp, u8p]
        L.orc_ppe_rhs.restype = C.c_int
        L.orc_ppe_rhs.argtypes = [C.c_int, C.c_int64, dp, dp, C.c_int, C.c_double, C.c_int, C.c_double, C.c_double,
                                  C.c_double, C.c_double, C.c_int, dp, dp, C.c_double, C.c_double, C.c_double, dp,
                                  u8p, dp, ip64, ip32, dp, dp, dp]
        L.orc_ppe_correct.restype = C.c_int
        L.orc_ppe_correct.argtypes = [C.c_int, C.c_int64, dp, dp, C.c_int, C.c_double, C.c_int, C.c_double,
                                      C.c_double, C.c_double, C.c_double, C.c_int, dp, dp, dp, C.c_double,
                                      C.c_double, ip64, ip32, dp]
        L.orc_ppe_bicgstab.restype = C.c_int
        L.orc_ppe_bicgstab.argtypes = [C.c_int64, ip64, ip32, dp, u8p, dp, dp, C.c_double, C.c_int,
                                       C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.orc_ops0.restype = C.c_int
        L.orc_ops0.argtypes = [C.c_int, C.c_int64, dp, dp, C.c_int, dp, C.c_int, C.c_double, C.c_int,
                               C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, dp, C.c_int64, ip64,
                               ip64, ip32, dp, u8p]
        L.orc_lap0.restype = C.c_int
        L.orc_lap0.argtypes = [C.c_int, C.c_int64, dp, dp, C.c_int, dp, C.c_int, C.c_double, C.c_int64, ip64,
                               ip64, ip32, dp]
        L.orc_grad_sum.restype = C.c_int
        L.orc_grad_sum.argtypes = [C.c_int, C.c_int64, dp, dp, dp, C.c_double, dp, C.c_int, C.c_double, C.c_int,
                                   C.c_double, C.c_double, C.c_double, C.c_double, C.c_int, dp, C.c_int64, ip64,
                                   ip64, ip32, dp, u8p]
        L.orc_threads.restype = C.c_int
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _p(a, t=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


_PP_KEEP = None   # the per-particle table the library points at


def _map_args(ms):
    """The mapping as C arguments; a per-particle table (kind 5, ms.pp of
    shape (12, n) in the particles' order) is handed to the library first."""
    global _PP_KEEP
    if int(ms.kind) == 5:
        _PP_KEEP = _f64(ms.pp)
        if _PP_KEEP.ndim != 2 or _PP_KEEP.shape[0] != 12:
            raise ValueError("per-particle map: pp must be (12, n)")
        lib().orc_set_per_particle(_p(_PP_KEEP), _PP_KEEP.shape[1])
    else:
        _PP_KEEP = None
        lib().orc_set_per_particle(None, 0)
    terms = _f64(ms.as_array())
    return (int(ms.kind), float(ms.Hhat), float(ms.H), float(ms.dmin), float(ms.eps),
            int(terms.shape[0]), terms)


def threads():
    return lib().orc_threads()


def set_threads(n):
    """OpenMP threads of the following oracle calls (for timing)."""
    lib().orc_set_threads(int(n))


def kernel_eval(kernel, dim, R, r):
    w, dw = C.c_double(), C.c_double()
    lib().orc_kernel_eval(int(kernel), int(dim), float(R), float(r), C.byref(w), C.byref(dw))
    return w.value, dw.value


def neighbors(pos, R, rows=None, brute=False):
    """CSR neighbour lists (original indices, ascending) of the given rows."""
    pos = _f64(pos)
    dim, n = pos.shape
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = n if rows_a is None else rows_a.shape[0]
    row_ptr = np.zeros(nr + 1, dtype=np.int64)
    nnz = lib().orc_neighbors(dim, n, _p(pos), float(R), nr, _p(rows_a, C.c_int64), int(brute),
                              _p(row_ptr, C.c_int64), None, 0)
    if nnz < 0:
        raise RuntimeError(f"orc_neighbors failed ({nnz})")
    col = np.zeros(max(nnz, 1), dtype=np.int32)
    nnz2 = lib().orc_neighbors(dim, n, _p(pos), float(R), nr, _p(rows_a, C.c_int64), int(brute),
                               _p(row_ptr, C.c_int64), _p(col, C.c_int32), col.shape[0])
    assert nnz2 == nnz
    return row_ptr, col[:nnz]


def sph2(pos, vol, phi, kernel, R, mapspec, rows=None, csr=None, grad_order=2):
    """Per-particle SPH(2) records (nrows, nf, REC) and flags (nrows,)."""
    pos = _f64(pos)
    vol = _f64(vol)
    phi = _f64(np.atleast_2d(phi))
    dim, n = pos.shape
    nf = phi.shape[0]
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    if csr is None:
        csr = neighbors(pos, R, rows=rows_a)
    row_ptr, col = csr
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    nr = n if rows_a is None else rows_a.shape[0]
    out = np.zeros((nr, nf, REC), dtype=np.float64)
    flags = np.zeros(nr, dtype=np.uint8)
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    st = lib().orc_sph2(dim, n, _p(pos), _p(vol), nf, _p(phi), int(kernel), float(R), kind, Hh, H,
                        dmin, eps, nt, _p(terms), int(grad_order), nr, _p(rows_a, C.c_int64),
                        _p(row_ptr, C.c_int64), _p(col if col.size else np.zeros(1, np.int32), C.c_int32),
                        _p(out), _p(flags, C.c_uint8))
    if st != 0:
        raise RuntimeError(f"orc_sph2 failed ({st})")
    return out, flags


def adjoint_dphi(pos, vol, kernel, R, mapspec, u, ks=None, csr=None, grad_order=2):
    """dphi_k = sum_i u_i d(lap_i)/d(phi_k) at sampled k (all if ks is None)."""
    pos = _f64(pos)
    vol = _f64(vol)
    u = _f64(u)
    dim, n = pos.shape
    if csr is None:
        csr = neighbors(pos, R)
    row_ptr, col = csr
    ks_a = None if ks is None else np.ascontiguousarray(ks, dtype=np.int64)
    nk = n if ks_a is None else ks_a.shape[0]
    out = np.zeros(nk, dtype=np.float64)
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    st = lib().orc_adjoint_dphi(dim, n, _p(pos), _p(vol), int(kernel), float(R), kind, Hh, H, dmin,
                                eps, nt, _p(terms), int(grad_order),
                                _p(np.ascontiguousarray(row_ptr, dtype=np.int64), C.c_int64),
                                _p(np.ascontiguousarray(col, dtype=np.int32), C.c_int32), _p(u), nk,
                                _p(ks_a, C.c_int64), _p(out))
    if st != 0:
        raise RuntimeError("orc_adjoint_dphi failed")
    return out


def dtheta(pos, mapspec, u, dhat, tlist):
    """sum_i u_i d(c_trans_i)/d(coef_t) . Dhat_i for each term index t."""
    pos = _f64(pos)
    dim, n = pos.shape
    u = _f64(u)
    dhat = _f64(dhat).reshape(n, 6)
    tl = np.ascontiguousarray(tlist, dtype=np.int32)
    out = np.zeros(tl.shape[0], dtype=np.float64)
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    lib().orc_dtheta(dim, n, _p(pos), kind, Hh, H, dmin, eps, nt, _p(terms), _p(u), _p(dhat),
                     tl.shape[0], _p(tl, C.c_int32), _p(out))
    return out


def map_eval(dim, x, y, zh, mapspec, t=-1):
    """(np, 24): J (9), c_trans (6), second derivatives of z^ (9); or their
    complex-step derivative with respect to term t."""
    x = _f64(x)
    zh = _f64(zh)
    y = None if y is None else _f64(y)
    out = np.zeros((x.shape[0], 24))
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    lib().orc_map_eval(dim, x.shape[0], _p(x), _p(y), _p(zh), kind, Hh, H, dmin, eps, nt, _p(terms),
                       int(t), _p(out))
    return out


def alpha_beta(dim, x, y, mapspec):
    x = _f64(x)
    y = None if y is None else _f64(y)
    out = np.zeros((x.shape[0], 12))
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    lib().orc_alpha_beta(dim, x.shape[0], _p(x), _p(y), kind, Hh, H, dmin, eps, nt, _p(terms), _p(out))
    return out


# ---------------------------------------------------------------- ISPH pressure step (Sec. 3.3)

def _csr(pos, R, csr):
    if csr is None:
        csr = neighbors(pos, R)
    rp, col = csr
    return np.ascontiguousarray(rp, dtype=np.int64), np.ascontiguousarray(col, dtype=np.int32)


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def lap_weights(pos, vol, kernel, R, mapspec, csr=None, grad_order=2):
    """Weights W (CSR layout of `csr`) of the physical Laplacian,
    lap_i = sum_j W_ij (phi_j - phi_i), and per-particle flags."""
    pos, vol = _f64(pos), _f64(vol)
    dim, n = pos.shape
    rp, col = _csr(pos, R, csr)
    W = np.zeros(max(col.shape[0], 1))
    flags = np.zeros(n, dtype=np.uint8)
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    st = lib().orc_lap_weights(dim, n, _p(pos), _p(vol), int(kernel), float(R), kind, Hh, H, dmin, eps, nt,
                               _p(terms), int(grad_order), n, None, _p(rp, C.c_int64),
                               _p(col if col.size else np.zeros(1, np.int32), C.c_int32), _p(W), _p(flags, C.c_uint8))
    if st != 0:
        raise RuntimeError("orc_lap_weights failed")
    return (rp, col, W[: col.shape[0]]), flags


def ppe_rhs(pos, vol, kernel, R, mapspec, v, rho, dt, gamma, jr=None, dirichlet=None, pbc=None, csr=None):
    """(rhs, div, dens) of the pressure Poisson equation."""
    pos, vol, v = _f64(pos), _f64(vol), _f64(v)
    dim, n = pos.shape
    rp, col = _csr(pos, R, csr)
    rhs, div, dens = np.zeros(n), np.zeros(n), np.zeros(n)
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    jr_a = None if jr is None else _f64(jr)
    pbc_a = None if pbc is None else _f64(pbc)
    dir_a = _u8(dirichlet)
    st = lib().orc_ppe_rhs(dim, n, _p(pos), _p(vol), int(kernel), float(R), kind, Hh, H, dmin, eps, nt, _p(terms),
                           _p(v), float(rho), float(dt), float(gamma), _p(jr_a), _p(dir_a, C.c_uint8), _p(pbc_a),
                           _p(rp, C.c_int64), _p(col if col.size else np.zeros(1, np.int32), C.c_int32), _p(rhs),
                           _p(div), _p(dens))
    if st != 0:
        raise RuntimeError("orc_ppe_rhs failed")
    return rhs, div, dens


def ppe_correct(pos, vol, kernel, R, mapspec, p, vstar, rho, dt, csr=None):
    """v* - dt / rho * (physical first-order pressure gradient), (dim, n)."""
    pos, vol, p, vstar = _f64(pos), _f64(vol), _f64(p), _f64(vstar)
    dim, n = pos.shape
    rp, col = _csr(pos, R, csr)
    out = np.zeros((dim, n))
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    st = lib().orc_ppe_correct(dim, n, _p(pos), _p(vol), int(kernel), float(R), kind, Hh, H, dmin, eps, nt,
                               _p(terms), _p(p), _p(vstar), float(rho), float(dt), _p(rp, C.c_int64),
                               _p(col if col.size else np.zeros(1, np.int32), C.c_int32), _p(out))
    if st != 0:
        raise RuntimeError("orc_ppe_correct failed")
    return out


def ppe_matvec(weights, dirichlet, x):
    """A x of the pressure system (numpy, for checks)."""
    rp, col, W = weights
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    y = np.zeros(n)
    np.add.at(y, rows, W * (x[col] - x[rows]))
    if dirichlet is not None:
        d = np.asarray(dirichlet, dtype=bool)
        y[d] = x[d]
    return y


def ppe_bicgstab(weights, dirichlet, b, x0=None, tol=1e-10, maxit=2000):
    """BiCGSTAB on the pressure system; returns (x, iterations, relres, status)."""
    rp, col, W = weights
    n = rp.shape[0] - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    b = _f64(b)
    it, rr = C.c_int(0), C.c_double(0.0)
    st = lib().orc_ppe_bicgstab(n, _p(rp, C.c_int64), _p(col if col.size else np.zeros(1, np.int32), C.c_int32),
                                _p(_f64(W)), _p(_u8(dirichlet), C.c_uint8), _p(b), _p(x), float(tol), int(maxit),
                                C.byref(it), C.byref(rr))
    return x, it.value, rr.value, st


# ------------------------------------------------------ conventional ISPH operators


def _rows_csr(pos, R, rows, csr):
    n = pos.shape[1]
    rows_a = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    if csr is None:
        csr = neighbors(pos, R, rows=rows_a)
    row_ptr = np.ascontiguousarray(csr[0], dtype=np.int64)
    col = np.ascontiguousarray(csr[1], dtype=np.int32)
    if col.size == 0:
        col = np.zeros(1, np.int32)
    nr = n if rows_a is None else rows_a.shape[0]
    return rows_a, row_ptr, col, nr


def ops0(pos, vol, phi, kernel, R, mapspec, rows=None, csr=None):
    """0th-order operator records (Sec. 3.1, Eq. sec_0th) through the map:
    (nrows, nf, REC) in sph2()'s layout, and flags (nrows,)."""
    pos, vol = _f64(pos), _f64(vol)
    phi = _f64(np.atleast_2d(phi))
    dim, n = pos.shape
    nf = phi.shape[0]
    rows_a, row_ptr, col, nr = _rows_csr(pos, R, rows, csr)
    out = np.zeros((nr, nf, REC))
    flags = np.zeros(nr, dtype=np.uint8)
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    st = lib().orc_ops0(dim, n, _p(pos), _p(vol), nf, _p(phi), int(kernel), float(R), kind, Hh, H, dmin, eps,
                        nt, _p(terms), nr, _p(rows_a, C.c_int64), _p(row_ptr, C.c_int64), _p(col, C.c_int32),
                        _p(out), _p(flags, C.c_uint8))
    if st != 0:
        raise RuntimeError(f"orc_ops0 failed ({st})")
    return out, flags


def lap0(pos, vol, phi, kernel, R, rows=None, csr=None):
    """The 0th-order (Brookshaw) Laplacian in the projected space, (nrows, nf)."""
    pos, vol = _f64(pos), _f64(vol)
    phi = _f64(np.atleast_2d(phi))
    dim, n = pos.shape
    nf = phi.shape[0]
    rows_a, row_ptr, col, nr = _rows_csr(pos, R, rows, csr)
    out = np.zeros((nr, nf))
    st = lib().orc_lap0(dim, n, _p(pos), _p(vol), nf, _p(phi), int(kernel), float(R), nr, _p(rows_a, C.c_int64),
                        _p(row_ptr, C.c_int64), _p(col, C.c_int32), _p(out))
    if st != 0:
        raise RuntimeError(f"orc_lap0 failed ({st})")
    return out


def grad_sum(pos, vol, p, kernel, R, mapspec, rho=None, rho0=1.0, rows=None, csr=None):
    """Summation pressure gradient (Eq. gra_sum): physical (nrows, 3),
    projected (nrows, 3) in the 3-D slot order, flags (nrows,)."""
    pos, vol, p = _f64(pos), _f64(vol), _f64(p)
    rho_a = None if rho is None else _f64(rho)
    dim, n = pos.shape
    rows_a, row_ptr, col, nr = _rows_csr(pos, R, rows, csr)
    out = np.zeros((nr, 6))
    flags = np.zeros(nr, dtype=np.uint8)
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    st = lib().orc_grad_sum(dim, n, _p(pos), _p(vol), _p(rho_a), float(rho0), _p(p), int(kernel), float(R), kind,
                            Hh, H, dmin, eps, nt, _p(terms), nr, _p(rows_a, C.c_int64), _p(row_ptr, C.c_int64),
                            _p(col, C.c_int32), _p(out), _p(flags, C.c_uint8))
    if st != 0:
        raise RuntimeError(f"orc_grad_sum failed ({st})")
    return out[:, :3], out[:, 3:], flags


# ------------------------------------------------------ volume smoothing (Sec. 3.6)


def jbar_smooth(pos, J, jbar, cv, re, order=None, csr=None):
    """Jbar^N from Jbar^(N-1) by Eq. VCT_bar_a, sequentially: targets in
    `order` (index order if None), the neighbours of each in the order of its
    CSR row (`csr` in original indices; the oracle's grid search if None)."""
    pos = _f64(pos)
    dim, n = pos.shape
    rp, col = _csr(pos, re, csr)
    out = _f64(jbar).copy()
    order_a = None if order is None else np.ascontiguousarray(order, dtype=np.int64)
    if order_a is not None and (order_a.shape != (n,) or not np.array_equal(np.sort(order_a), np.arange(n))):
        raise ValueError("order must be a permutation of the particles")
    st = lib().orc_jbar_smooth(dim, n, _p(pos), _p(_f64(J)), _p(out), float(cv), float(re), _p(order_a, C.c_int64),
                               _p(rp, C.c_int64), _p(col if col.size else np.zeros(1, np.int32), C.c_int32))
    if st != 0:
        raise RuntimeError("orc_jbar_smooth failed")
    return out


# ------------------------------------------------ bathymetry adjoint, reading R2


def project(phys, mapspec):
    """Projected positions of physical points (dim, n): z^ = alpha (z + beta)."""
    phys = _f64(phys)
    dim, n = phys.shape
    out = np.zeros_like(phys)
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    lib().orc_project(dim, n, _p(phys), kind, Hh, H, dmin, eps, nt, _p(terms), _p(out))
    return out


def r2_dzhat(pos, vol, phi, kernel, R, mapspec, u, ks=None, csr=None, ct_dep=True):
    """d loss / d z^_k (loss = sum (lap - g)^2, u = 2 (lap - g)) at sampled
    particles, by the complex step of z^_k; ct_dep=False holds c_trans."""
    pos, vol, phi, u = _f64(pos), _f64(vol), _f64(phi).reshape(-1), _f64(u)
    dim, n = pos.shape
    rp, col = _csr(pos, R, csr)
    ks_a = None if ks is None else np.ascontiguousarray(ks, dtype=np.int64)
    nk = n if ks_a is None else ks_a.shape[0]
    out = np.zeros(nk)
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    st = lib().orc_r2_dzhat(dim, n, _p(pos), _p(vol), _p(phi), int(kernel), float(R), kind, Hh, H, dmin, eps, nt,
                            _p(terms), _p(u), int(bool(ct_dep)), nk, _p(ks_a, C.c_int64), _p(rp, C.c_int64),
                            _p(col if col.size else np.zeros(1, np.int32), C.c_int32), _p(out))
    if st != 0:
        raise RuntimeError("orc_r2_dzhat failed")
    return out


def r2_dtheta(phys, vol, phi, g, kernel, R, mapspec, tlist, csr):
    """d loss / d coef_t with physical positions fixed (reading R2), by the
    complex step through the whole evaluation; csr: neighbour lists of the
    projected positions (original indices)."""
    phys, vol, phi, g = _f64(phys), _f64(vol), _f64(phi).reshape(-1), _f64(g)
    dim, n = phys.shape
    rp, col = np.ascontiguousarray(csr[0], dtype=np.int64), np.ascontiguousarray(csr[1], dtype=np.int32)
    tl = np.ascontiguousarray(tlist, dtype=np.int32)
    out = np.zeros(tl.shape[0])
    kind, Hh, H, dmin, eps, nt, terms = _map_args(mapspec)
    st = lib().orc_r2_dtheta(dim, n, _p(phys), _p(vol), _p(phi), _p(g), int(kernel), float(R), kind, Hh, H, dmin,
                             eps, nt, _p(terms), tl.shape[0], _p(tl, C.c_int32), _p(rp, C.c_int64),
                             _p(col if col.size else np.zeros(1, np.int32), C.c_int32), _p(out))
    if st != 0:
        raise RuntimeError("orc_r2_dtheta failed")
    return out
