"""Python binding of libvct (ctypes): argument marshalling only.

Every computation runs in the HIP kernels of libvct.so.  PyTorch supplies
device memory and the current stream.  If the shared library has not been
built, every call raises (there is no CPU fallback).

Functions named like the C ABI (vct_*) take torch tensors (device) and plain
Python numbers, pass raw pointers and the current HIP stream, and raise
VctError on negative status.  `Geometry` strings the calls together for one
particle set: cell sort, neighbour lists, moments, and repeated applies.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvct.so")

VCT_OK, VCT_W_FLAGGED, VCT_W_NOCONV = 0, 1, 2
VCT_E_ARG, VCT_E_HIP, VCT_E_CAPACITY, VCT_E_NONFINITE, VCT_E_WORKSPACE, VCT_E_WINDOW = -1, -2, -3, -4, -5, -6
VCT_KERNEL_WENDLAND_C2, VCT_KERNEL_CUBIC_SPLINE = 0, 1
VCT_FP64, VCT_MIXED, VCT_MIXED_S64 = 0, 1, 2
VCT_OUT_GRAD, VCT_OUT_LAP, VCT_OUT_CROSS, VCT_OUT_HESS, VCT_OUT_PGRAD, VCT_OUT_PHESS = 1, 2, 4, 8, 16, 32
VCT_OUT_PZ = 64
VCT_OPT_GRAD1 = 256
VCT_OUT_DEFAULT = VCT_OUT_GRAD | VCT_OUT_LAP | VCT_OUT_CROSS
VCT_MAX_TERMS = 32
VCT_MAP_PER_PARTICLE = 5
FLAG_FEW, FLAG_SINGULAR_A, FLAG_SINGULAR_M, FLAG_NONFINITE, FLAG_DUPLICATE, FLAG_MAP = 1, 2, 4, 8, 16, 32


class VctError(RuntimeError):
    def __init__(self, name, status, detail=""):
        self.status = status
        super().__init__(f"{name}: {status_string(status)}" + (f" ({detail})" if detail else ""))


class vct_term(C.Structure):
    _fields_ = [("coef", C.c_double), ("bx", C.c_int32), ("by", C.c_int32), ("fx", C.c_double),
                ("fy", C.c_double)]


class vct_map(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nterms", C.c_int32), ("Hhat", C.c_double), ("H", C.c_double),
                ("dmin", C.c_double), ("eps", C.c_double), ("terms", C.POINTER(vct_term)), ("coef", C.c_void_p),
                ("coef_n", C.c_int64)]


class vct_nlist(C.Structure):
    _fields_ = [("dim", C.c_int32), ("reserved", C.c_int32), ("n", C.c_int64), ("ncell", C.c_int64),
                ("chunk_cap", C.c_int64), ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("R", C.c_double),
                ("cell_start", C.c_void_p), ("chunk_off", C.c_void_p), ("chunk_start", C.c_void_p),
                ("chunk_info", C.c_void_p), ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("col16", C.c_void_p),
                ("col_t", C.c_void_p), ("nnz", C.c_int64), ("chunk_win", C.c_void_p)]


_lib = None
_vp, _i64, _sz, _dp = C.c_void_p, C.c_int64, C.c_size_t, C.POINTER(C.c_double)
_nlp = C.POINTER(vct_nlist)


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("VCT_LIB") or LIB_PATH
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build() "
                               "(the operators have no CPU fallback)")
        L = C.CDLL(path)
        L.vct_status_string.restype = C.c_char_p
        L.vct_status_string.argtypes = [C.c_int]
        L.vct_last_error.restype = C.c_char_p
        L.vct_last_error.argtypes = []
        L.vct_grid_dims.restype = _i64
        L.vct_grid_dims.argtypes = [C.c_int, _dp, _dp, C.c_double, C.POINTER(_i64)]
        L.vct_n_out.restype = C.c_int
        L.vct_n_out.argtypes = [C.c_int, C.c_uint32]
        L.vct_state_stride.restype = C.c_int
        L.vct_state_stride.argtypes = [C.c_int, C.c_uint32]
        L.vct_build_cells_workspace_size.restype = _sz
        L.vct_build_cells_workspace_size.argtypes = [C.c_int, _i64, _i64]
        L.vct_build_cells.restype = C.c_int
        L.vct_build_cells.argtypes = [C.c_int, _i64, _vp, _dp, _dp, C.c_double, _vp, _vp, _vp, _i64, _vp, _sz,
                                      _vp]
        L.vct_gather_sorted.restype = C.c_int
        L.vct_gather_sorted.argtypes = [_i64, C.c_int, _vp, _vp, _vp, _vp]
        L.vct_scatter_sorted.restype = C.c_int
        L.vct_scatter_sorted.argtypes = [_i64, C.c_int, _vp, _vp, _vp, _vp]
        L.vct_chunk_capacity.restype = _i64
        L.vct_chunk_capacity.argtypes = [C.c_int, _i64, _i64]
        L.vct_timing_enable.restype = C.c_int
        L.vct_timing_enable.argtypes = [C.c_int]
        L.vct_device_checks.restype = C.c_int
        L.vct_device_checks.argtypes = [C.POINTER(C.c_uint32)]
        L.vct_timing_reset.restype = None
        L.vct_timing_reset.argtypes = []
        L.vct_timing_count.restype = C.c_int
        L.vct_timing_count.argtypes = []
        L.vct_timing_get.restype = C.c_int
        L.vct_timing_get.argtypes = [C.c_int, C.POINTER(C.c_char_p), C.POINTER(_i64), C.POINTER(C.c_double)]
        L.vct_neighbors_workspace_size.restype = _sz
        L.vct_neighbors_workspace_size.argtypes = [_i64, _i64]
        L.vct_neighbors.restype = C.c_int
        L.vct_neighbors.argtypes = [_nlp, _vp, _i64, C.POINTER(_i64), C.c_int, _vp, _sz, _vp]
        L.vct_moments_workspace_size.restype = _sz
        L.vct_moments_workspace_size.argtypes = [C.c_int, _i64]
        L.vct_moments.restype = C.c_int
        L.vct_moments.argtypes = [_nlp, _vp, _vp, C.c_int, C.POINTER(vct_map), C.c_uint32, _vp, _vp, _vp,
                                  C.POINTER(_i64), _vp, _sz, _vp]
        L.vct_moments_ex.restype = C.c_int
        L.vct_moments_ex.argtypes = [_nlp, _vp, _vp, C.c_int, C.POINTER(vct_map), C.c_uint32, _vp, _vp, C.c_uint32,
                                     _vp, _vp, _vp, C.POINTER(_i64), _vp, _sz, _vp]
        L.vct_moments_resolve.restype = C.c_int
        L.vct_moments_resolve.argtypes = [_nlp, _vp, C.POINTER(vct_map), C.c_uint32, _vp, _vp, _vp,
                                          C.POINTER(_i64), _vp, _sz, _vp]
        L.vct_apply_ops.restype = C.c_int
        L.vct_apply_ops.argtypes = [_nlp, C.c_int, _vp, _vp, _vp, C.c_int, _vp, C.c_uint32, C.c_int, _vp, _vp]
        L.vct_apply_ops_ex.restype = C.c_int
        L.vct_apply_ops_ex.argtypes = [_nlp, C.c_int, _vp, _vp, _vp, C.c_int, _vp, C.c_uint32, C.c_int, _vp, _vp, _vp,
                                       _vp]
        L.vct_adjoint_workspace_size.restype = _sz
        L.vct_adjoint_workspace_size.argtypes = [C.c_int, _i64, _i64, C.c_int]
        L.vct_apply_ops_adjoint.restype = C.c_int
        L.vct_apply_ops_adjoint.argtypes = [_nlp, _vp, _vp, C.c_int, _vp, C.c_uint32, C.POINTER(vct_map), _vp, _vp,
                                            _vp, _vp, _vp, _sz, _vp]
        L.vct_ppe_rhs.restype = C.c_int
        L.vct_ppe_rhs.argtypes = [_nlp, _vp, _vp, C.c_int, _vp, C.c_uint32, C.POINTER(vct_map), _vp, C.c_double,
                                  C.c_double, C.c_double, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.vct_ppe_correct.restype = C.c_int
        L.vct_ppe_correct.argtypes = [_nlp, _vp, _vp, C.c_int, _vp, C.c_uint32, C.POINTER(vct_map), _vp, _vp,
                                      C.c_double, C.c_double, _vp, _vp]
        L.vct_ppe_workspace_size.restype = _sz
        L.vct_ppe_workspace_size.argtypes = [C.c_int, _i64, C.c_uint32]
        L.vct_ppe_solve.restype = C.c_int
        L.vct_ppe_solve.argtypes = [_nlp, _vp, _vp, C.c_int, _vp, C.c_uint32, _vp, _vp, _vp, C.c_double, C.c_int,
                                    C.POINTER(C.c_int), C.POINTER(C.c_double), _vp, _sz, _vp]
        L.vct_apply_ops0.restype = C.c_int
        L.vct_apply_ops0.argtypes = [_nlp, C.c_int, _vp, _vp, _vp, C.c_int, C.POINTER(vct_map), C.c_uint32, _vp, _vp]
        L.vct_grad_sum.restype = C.c_int
        L.vct_grad_sum.argtypes = [_nlp, _vp, _vp, C.c_int, C.POINTER(vct_map), _vp, C.c_double, _vp, C.c_uint32,
                                   _vp, _vp]
        L.vct_apply_ops_adjoint_noalloc.restype = C.c_int
        L.vct_apply_ops_adjoint_noalloc.argtypes = [_nlp, _vp, _vp, C.c_int, _vp, C.c_uint32, C.POINTER(vct_map), _vp,
                                                    _vp, _vp, _vp, _vp]
        L.vct_map_alpha.restype = C.c_int
        L.vct_map_alpha.argtypes = [C.c_int, _i64, _vp, C.POINTER(vct_map), _vp, _vp]
        L.vct_adjoint_r2_workspace_size.restype = _sz
        L.vct_adjoint_r2_workspace_size.argtypes = [C.c_int, _i64, C.c_int]
        L.vct_apply_ops_adjoint_r2.restype = C.c_int
        L.vct_apply_ops_adjoint_r2.argtypes = [_nlp, _vp, _vp, C.c_int, _vp, C.c_uint32, C.POINTER(vct_map), _vp,
                                               _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.vct_map_project.restype = C.c_int
        L.vct_map_project.argtypes = [C.c_int, _i64, _vp, C.POINTER(vct_map), _vp, _vp]
        L.vct_jbar_workspace_size.restype = _sz
        L.vct_jbar_workspace_size.argtypes = [_i64]
        L.vct_jbar_smooth.restype = C.c_int
        L.vct_jbar_smooth.argtypes = [_nlp, _vp, _vp, _vp, C.c_double, C.c_double, _vp, _sz, _vp]
        _lib = L
    return _lib


def status_string(st):
    return lib().vct_status_string(int(st)).decode()


def _check(name, st):
    if st < 0:
        detail = lib().vct_last_error().decode() if st == VCT_E_HIP else ""
        raise VctError(name, st, detail)
    return st


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _d3(v):
    a = (C.c_double * 3)()
    for k, x in enumerate(list(v)[:3]):
        a[k] = float(x)
    return a


def make_map(mapspec, coef=None):
    """vct_map (plus the term array it points to) from an inputs.MapSpec; for
    the per-particle kind, `coef` is the (12, n) FP64 device table in the
    order of the call's points."""
    terms = mapspec.as_array()
    nt = terms.shape[0]
    if nt > VCT_MAX_TERMS:
        raise ValueError(f"at most {VCT_MAX_TERMS} bathymetry terms")
    arr = (vct_term * max(nt, 1))()
    for t in range(nt):
        arr[t] = vct_term(float(terms[t, 0]), int(terms[t, 1]), int(terms[t, 3]), float(terms[t, 2]),
                          float(terms[t, 4]))
    m = vct_map(int(mapspec.kind), nt, float(mapspec.Hhat), float(mapspec.H), float(mapspec.dmin),
                float(mapspec.eps), C.cast(arr, C.POINTER(vct_term)), None, 0)
    if coef is not None:
        if coef.dtype != __import__("torch").float64 or not coef.is_contiguous() or coef.dim() != 2 \
                or coef.shape[0] != 12:
            raise ValueError("per-particle coefficients: a contiguous (12, n) float64 tensor")
        m.coef, m.coef_n = coef.data_ptr(), int(coef.shape[1])
    m._keep = (arr, coef)
    return m


# ---------------------------------------------------------------- thin wrappers

def vct_grid_dims(dim, lo, hi, R):
    dims = (_i64 * 3)()
    nc = lib().vct_grid_dims(dim, _d3(lo), _d3(hi), float(R), dims)
    _check("vct_grid_dims", nc if nc < 0 else 0)
    return int(nc), tuple(dims)


def vct_n_out(dim, mask):
    return lib().vct_n_out(dim, mask)


def vct_state_stride(dim, mask):
    return lib().vct_state_stride(dim, mask)


def vct_build_cells(dim, n, pos, lo, hi, R, perm, pos_sorted, cell_start, ncell, ws, stream=None):
    return _check("vct_build_cells", lib().vct_build_cells(
        dim, n, _p(pos), _d3(lo), _d3(hi), float(R), _p(perm), _p(pos_sorted), _p(cell_start), ncell, _p(ws),
        _nbytes(ws), _stream(stream)))


def vct_gather_sorted(n, ncomp, perm, src, dst, stream=None):
    return _check("vct_gather_sorted", lib().vct_gather_sorted(n, ncomp, _p(perm), _p(src), _p(dst),
                                                                _stream(stream)))


def vct_scatter_sorted(n, ncomp, perm, src, dst, stream=None):
    return _check("vct_scatter_sorted", lib().vct_scatter_sorted(n, ncomp, _p(perm), _p(src), _p(dst),
                                                                  _stream(stream)))


def _nbytes(t):
    return 0 if t is None else t.numel() * t.element_size()


def make_nlist(dim, n, ncell, lo, hi, R, cell_start, chunk_off, chunk_start, chunk_info, row_ptr, col=None,
               col16=None, chunk_cap=None, col_t=None, chunk_win=None):
    """vct_nlist over torch tensors (device)."""
    nl = vct_nlist()
    nl.dim, nl.n, nl.ncell = int(dim), int(n), int(ncell)
    nl.chunk_cap = int(chunk_cap if chunk_cap is not None else chunk_start.numel() - 1)
    for k in range(3):
        nl.lo[k] = float(lo[k]) if k < len(lo) else 0.0
        nl.hi[k] = float(hi[k]) if k < len(hi) else 0.0
    nl.R = float(R)
    nl.cell_start, nl.chunk_off, nl.chunk_start = cell_start.data_ptr(), chunk_off.data_ptr(), chunk_start.data_ptr()
    nl.chunk_info, nl.row_ptr = chunk_info.data_ptr(), row_ptr.data_ptr()
    nl.col = col.data_ptr() if col is not None else None
    nl.col16 = col16.data_ptr() if col16 is not None else None
    nl.col_t = col_t.data_ptr() if col_t is not None else None
    nl.chunk_win = chunk_win.data_ptr() if chunk_win is not None else None
    return nl


def vct_timing_enable(on):
    return lib().vct_timing_enable(int(bool(on)))


VCT_CHECK_WINDOW, VCT_CHECK_CAPACITY, VCT_CHECK_ACCUM = 1, 2, 4


def vct_device_checks():
    """(checked, bits): whether the loaded library is the debug build with
    device bounds checks, and the check bits set since the previous call
    (cleared by this call; waits for the device)."""
    bits = C.c_uint32(0)
    st = lib().vct_device_checks(C.byref(bits))
    if st < 0:
        _check("vct_device_checks", st)
    return bool(st), int(bits.value)


def vct_timing_reset():
    lib().vct_timing_reset()


def vct_timing_read():
    """{kernel name: (launches, summed ms)} of the launches timed so far."""
    L = lib()
    res = {}
    for k in range(L.vct_timing_count()):
        nm, cnt, ms = C.c_char_p(), _i64(0), C.c_double(0.0)
        _check("vct_timing_get", L.vct_timing_get(k, C.byref(nm), C.byref(cnt), C.byref(ms)))
        res[nm.value.decode()] = (cnt.value, ms.value)
    return res


def vct_neighbors(nl, pos_sorted, col_cap, reuse, ws, stream=None):
    nnz = _i64(0)
    st = lib().vct_neighbors(C.byref(nl), _p(pos_sorted), int(col_cap), C.byref(nnz), int(reuse), _p(ws),
                             _nbytes(ws), _stream(stream))
    if st == VCT_E_CAPACITY:
        return st, nnz.value
    _check("vct_neighbors", st)
    return st, nnz.value


def vct_moments(nl, pos_sorted, vol_sorted, kernel, cmap, mask, state64, state32, flags, count_flagged, ws,
                stream=None):
    cnt = _i64(0)
    st = lib().vct_moments(C.byref(nl), _p(pos_sorted), _p(vol_sorted), kernel, C.byref(cmap), mask, _p(state64),
                           _p(state32), _p(flags), C.byref(cnt) if count_flagged else None, _p(ws), _nbytes(ws),
                           _stream(stream))
    _check("vct_moments", st)
    return st, cnt.value


def vct_moments_ex(nl, pos_sorted, vol_sorted, kernel, cmap, mask, state64, state32, mask2, state64_2, state32_2,
                   flags, count_flagged, ws, stream=None):
    """vct_moments folding the same inverse into a second state (mask2)."""
    cnt = _i64(0)
    st = lib().vct_moments_ex(C.byref(nl), _p(pos_sorted), _p(vol_sorted), kernel, C.byref(cmap), mask, _p(state64),
                              _p(state32), mask2, _p(state64_2), _p(state32_2), _p(flags),
                              C.byref(cnt) if count_flagged else None, _p(ws), _nbytes(ws), _stream(stream))
    _check("vct_moments_ex", st)
    return st, cnt.value


def vct_moments_resolve(nl, pos_sorted, cmap, mask, state64, state32, flags, count_flagged, ws, stream=None):
    cnt = _i64(0)
    st = lib().vct_moments_resolve(C.byref(nl), _p(pos_sorted), C.byref(cmap), mask, _p(state64), _p(state32),
                                   _p(flags), C.byref(cnt) if count_flagged else None, _p(ws), _nbytes(ws),
                                   _stream(stream))
    _check("vct_moments_resolve", st)
    return st, cnt.value


def vct_apply_ops(nl, nf, phi_sorted, pos_sorted, vol_sorted, kernel, state, mask, precision, out, stream=None):
    return _check("vct_apply_ops", lib().vct_apply_ops(
        C.byref(nl), nf, _p(phi_sorted), _p(pos_sorted), _p(vol_sorted), kernel, _p(state), mask, precision, _p(out),
        _stream(stream)))


def vct_apply_ops_ex(nl, nf, phi_sorted, pos_sorted, vol_sorted, kernel, state, mask, precision, out, g_out=None,
                     g_in=None, stream=None):
    """vct_apply_ops with the first pass's gradient G~ [nf][d][n] FP32 written
    to g_out, or (FP64 only) taken from g_in instead of computed."""
    return _check("vct_apply_ops_ex", lib().vct_apply_ops_ex(
        C.byref(nl), nf, _p(phi_sorted), _p(pos_sorted), _p(vol_sorted), kernel, _p(state), mask, precision, _p(out),
        _p(g_out), _p(g_in), _stream(stream)))


def vct_apply_ops_adjoint(nl, pos_sorted, vol_sorted, kernel, state64, mask, cmap, proj, u, dphi, dtheta, ws,
                          stream=None):
    return _check("vct_apply_ops_adjoint", lib().vct_apply_ops_adjoint(
        C.byref(nl), _p(pos_sorted), _p(vol_sorted), kernel, _p(state64), mask, C.byref(cmap), _p(proj), _p(u),
        _p(dphi), _p(dtheta), _p(ws), _nbytes(ws), _stream(stream)))


def vct_apply_ops_adjoint_noalloc(nl, pos_sorted, vol_sorted, kernel, state64, mask, cmap, proj, u, dphi, dtheta,
                                  stream=None):
    return _check("vct_apply_ops_adjoint_noalloc", lib().vct_apply_ops_adjoint_noalloc(
        C.byref(nl), _p(pos_sorted), _p(vol_sorted), kernel, _p(state64), mask, C.byref(cmap), _p(proj), _p(u),
        _p(dphi), _p(dtheta), _stream(stream)))


def vct_ppe_rhs(nl, pos_sorted, vol_sorted, kernel, state64, mask, cmap, vstar, rho, dt, gamma, jr, dirichlet, pbc,
                rhs, div=None, dens=None, stream=None):
    return _check("vct_ppe_rhs", lib().vct_ppe_rhs(
        C.byref(nl), _p(pos_sorted), _p(vol_sorted), kernel, _p(state64), mask, C.byref(cmap), _p(vstar), float(rho),
        float(dt), float(gamma), _p(jr), _p(dirichlet), _p(pbc), _p(rhs), _p(div), _p(dens), _stream(stream)))


def vct_ppe_correct(nl, pos_sorted, vol_sorted, kernel, state64, mask, cmap, p, vstar, rho, dt, vout, stream=None):
    return _check("vct_ppe_correct", lib().vct_ppe_correct(
        C.byref(nl), _p(pos_sorted), _p(vol_sorted), kernel, _p(state64), mask, C.byref(cmap), _p(p), _p(vstar),
        float(rho), float(dt), _p(vout), _stream(stream)))


def vct_ppe_solve(nl, pos_sorted, vol_sorted, kernel, state64, mask, dirichlet, rhs, p, tol, max_iter, ws,
                  stream=None):
    """Returns (status, iterations, relative residual)."""
    it, rr = C.c_int(0), C.c_double(0.0)
    st = lib().vct_ppe_solve(C.byref(nl), _p(pos_sorted), _p(vol_sorted), kernel, _p(state64), mask, _p(dirichlet),
                             _p(rhs), _p(p), float(tol), int(max_iter), C.byref(it), C.byref(rr), _p(ws),
                             _nbytes(ws), _stream(stream))
    _check("vct_ppe_solve", st)
    return st, it.value, rr.value


def vct_apply_ops0(nl, nf, phi_sorted, pos_sorted, vol_sorted, kernel, cmap, mask, out, stream=None):
    return _check("vct_apply_ops0", lib().vct_apply_ops0(
        C.byref(nl), int(nf), _p(phi_sorted), _p(pos_sorted), _p(vol_sorted), kernel, C.byref(cmap), mask, _p(out),
        _stream(stream)))


def vct_grad_sum(nl, pos_sorted, vol_sorted, kernel, cmap, rho, rho0, p, mask, out, stream=None):
    return _check("vct_grad_sum", lib().vct_grad_sum(
        C.byref(nl), _p(pos_sorted), _p(vol_sorted), kernel, C.byref(cmap), _p(rho), float(rho0), _p(p), mask,
        _p(out), _stream(stream)))


def vct_apply_ops_adjoint_r2(nl, pos_sorted, vol_sorted, kernel, state64, mask, cmap, proj, phi, u, dtheta, dzhat,
                             ws, stream=None):
    return _check("vct_apply_ops_adjoint_r2", lib().vct_apply_ops_adjoint_r2(
        C.byref(nl), _p(pos_sorted), _p(vol_sorted), kernel, _p(state64), mask, C.byref(cmap), _p(proj), _p(phi),
        _p(u), _p(dtheta), _p(dzhat), _p(ws), _nbytes(ws), _stream(stream)))


def vct_map_project(dim, n, phys, cmap, proj, stream=None):
    return _check("vct_map_project", lib().vct_map_project(int(dim), int(n), _p(phys), C.byref(cmap), _p(proj),
                                                           _stream(stream)))


def vct_map_alpha(dim, n, pos, cmap, alpha, stream=None):
    return _check("vct_map_alpha", lib().vct_map_alpha(int(dim), int(n), _p(pos), C.byref(cmap), _p(alpha),
                                                       _stream(stream)))


def vct_jbar_smooth(nl, pos_sorted, J, jbar, cv, re, ws, stream=None):
    return _check("vct_jbar_smooth", lib().vct_jbar_smooth(
        C.byref(nl), _p(pos_sorted), _p(J), _p(jbar), float(cv), float(re), _p(ws), _nbytes(ws), _stream(stream)))


# ---------------------------------------------------------------- orchestration

def _bytes(nbytes, device):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Geometry:
    """One particle set on the GPU: cell sort, neighbour lists, per-particle
    state.  Positions are projected coordinates (dim, n) in the caller's order;
    `perm` maps sorted -> original."""

    def __init__(self, pos, vol, lo, hi, R, kernel=VCT_KERNEL_WENDLAND_C2, device="cuda", keep_col=True):
        import torch
        pos = torch.as_tensor(pos, dtype=torch.float64, device=device).contiguous()
        vol = torch.as_tensor(vol, dtype=torch.float64, device=device).contiguous()
        self.dim, self.n = int(pos.shape[0]), int(pos.shape[1])
        self.lo, self.hi, self.R, self.kernel, self.device = tuple(lo), tuple(hi), float(R), int(kernel), device
        self.ncell, self.dims = vct_grid_dims(self.dim, lo, hi, R)
        n = self.n
        self.perm = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        self.pos = torch.empty((self.dim, max(n, 1)), dtype=torch.float64, device=device)
        self.cell_start = torch.empty(self.ncell + 1, dtype=torch.int64, device=device)
        ws = _bytes(lib().vct_build_cells_workspace_size(self.dim, n, self.ncell), device)
        vct_build_cells(self.dim, n, pos, lo, hi, R, self.perm, self.pos, self.cell_start, self.ncell, ws)
        self.vol = torch.empty(max(n, 1), dtype=torch.float64, device=device)
        if n:
            vct_gather_sorted(n, 1, self.perm, vol, self.vol)
        self.row_ptr = torch.empty(n + 1, dtype=torch.int64, device=device)
        ncols = self.dims[0] * self.dims[1] if self.dim == 3 else self.dims[0]
        cap = lib().vct_chunk_capacity(self.dim, n, self.ncell)
        self.chunk_off = torch.empty(ncols + 1, dtype=torch.int64, device=device)
        self.chunk_start = torch.empty(cap + 1, dtype=torch.int32, device=device)
        self.chunk_info = torch.empty((cap, 4), dtype=torch.int32, device=device)
        self.chunk_win = torch.empty((cap, 32), dtype=torch.int32, device=device)
        self._nws = _bytes(lib().vct_neighbors_workspace_size(n, self.ncell), device)
        nl = make_nlist(self.dim, n, self.ncell, lo, hi, R, self.cell_start, self.chunk_off, self.chunk_start,
                        self.chunk_info, self.row_ptr, chunk_cap=cap, chunk_win=self.chunk_win)
        _, nnz = vct_neighbors(nl, self.pos, 0, 0, self._nws)
        self.nnz = nnz
        self.col = torch.empty(max(nnz, 1), dtype=torch.int32, device=device) if keep_col else None
        self.col16 = torch.empty(max(nnz, 1), dtype=torch.uint16, device=device)
        # transposed-entry map, for the adjoint (needs the int32 columns)
        self.col_t = torch.empty(max(nnz, 1), dtype=torch.int32, device=device) if keep_col else None
        self.nl = make_nlist(self.dim, n, self.ncell, lo, hi, R, self.cell_start, self.chunk_off, self.chunk_start,
                             self.chunk_info, self.row_ptr, self.col, self.col16, chunk_cap=cap, col_t=self.col_t,
                             chunk_win=self.chunk_win)
        # one search that stages the hit words and expands them into rows
        # (falling back to the fill pass by itself when a window is wider than
        # the staged words can describe)
        _, nnz2 = vct_neighbors(self.nl, self.pos, max(nnz, 1), 0, self._nws)
        if nnz2 != nnz:
            raise VctError("vct_neighbors", VCT_E_HIP)
        self.state64 = self.state32 = self.flags = None
        self.mask = None

    def map_for(self, mapspec):
        """vct_map of a MapSpec for calls on this geometry: a per-particle
        table (mapspec.pp, (12, n) in the caller's order) goes to the device
        in sorted order."""
        if int(mapspec.kind) != VCT_MAP_PER_PARTICLE:
            return make_map(mapspec)
        return make_map(mapspec, self.sorted_field(mapspec.pp).contiguous())

    def sorted_field(self, phi):
        """(nf, n) field in the caller's order -> sorted order (device)."""
        import torch
        phi = torch.as_tensor(phi, dtype=torch.float64, device=self.device)
        phi = phi.reshape(-1, self.n).contiguous()
        out = torch.empty_like(phi)
        if self.n:
            vct_gather_sorted(self.n, phi.shape[0], self.perm, phi, out)
        return out

    def unsort(self, x):
        """Rows over sorted particles -> caller's order; x is (..., n, k) or (n,)."""
        import torch
        idx = self.perm.long()[: self.n]
        out = torch.empty_like(x)
        if x.dim() == 1:
            out[idx] = x
        else:
            out[..., idx, :] = x
        return out

    def moments(self, mapspec, mask=VCT_OUT_DEFAULT, fp32_copy=False, count_flagged=True, fp64=True):
        """Per-particle state for `mask`; fp64=False with fp32_copy=True keeps
        only the FP32 state (enough for the mixed apply)."""
        import torch
        n, dim = self.n, self.dim
        stride = vct_state_stride(dim, mask)
        self.cmap = self.map_for(mapspec)
        self.mask = mask
        self.state64 = torch.empty((stride, max(n, 1)), dtype=torch.float64, device=self.device) if fp64 else None
        self.state32 = torch.empty((stride, max(n, 1)), dtype=torch.float32, device=self.device) if fp32_copy else None
        self.flags = torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)
        self.ws_mom = ws = _bytes(lib().vct_moments_workspace_size(dim, n), self.device)
        st, nflag = vct_moments(self.nl, self.pos, self.vol, self.kernel, self.cmap, mask, self.state64, self.state32,
                                self.flags, count_flagged, ws)
        self.n_flagged = nflag
        return st

    def resolve(self, mapspec, mask=VCT_OUT_DEFAULT, fp32_copy=False, count_flagged=True, fp64=True, ws=None):
        """The state for another mask or map, solved from the moment sums the
        last moments() call kept in its workspace (or in `ws`, the workspace of
        an earlier call on this geometry); no sweep over the rows."""
        import torch
        ws = ws if ws is not None else getattr(self, "ws_mom", None)
        if ws is None:
            raise ValueError("resolve() needs an earlier moments() call")
        n, dim = self.n, self.dim
        stride = vct_state_stride(dim, mask)
        self.cmap = self.map_for(mapspec)
        self.mask = mask
        self.state64 = torch.empty((stride, max(n, 1)), dtype=torch.float64, device=self.device) if fp64 else None
        self.state32 = torch.empty((stride, max(n, 1)), dtype=torch.float32, device=self.device) if fp32_copy else None
        self.flags = torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)
        st, nflag = vct_moments_resolve(self.nl, self.pos, self.cmap, mask, self.state64, self.state32, self.flags,
                                        count_flagged, ws)
        self.n_flagged = nflag
        return st

    def apply(self, phi_sorted, precision=VCT_FP64, out=None):
        import torch
        nf = int(phi_sorted.shape[0])
        nout = vct_n_out(self.dim, self.mask)
        if out is None:
            out = torch.empty((nf, max(self.n, 1), nout), dtype=torch.float64, device=self.device)
        state = self.state32 if precision == VCT_MIXED else self.state64
        if state is None:
            raise ValueError("VCT_MIXED needs moments(..., fp32_copy=True)")
        vct_apply_ops(self.nl, nf, phi_sorted, self.pos, self.vol, self.kernel, state, self.mask, precision, out)
        return out

    def apply0(self, mapspec, phi_sorted, mask=VCT_OUT_DEFAULT, out=None):
        """The 0th-order operators (conventional ISPH) of nf sorted fields:
        (nf, n, n_out) FP64.  Needs no moments."""
        import torch
        nf = int(phi_sorted.shape[0])
        nout = vct_n_out(self.dim, mask)
        if out is None:
            out = torch.empty((nf, max(self.n, 1), nout), dtype=torch.float64, device=self.device)
        vct_apply_ops0(self.nl, nf, phi_sorted, self.pos, self.vol, self.kernel, self.map_for(mapspec), mask, out)
        return out

    def grad_sum(self, mapspec, p_sorted, rho_sorted=None, rho0=1.0, mask=VCT_OUT_GRAD | VCT_OUT_PGRAD):
        """Summation pressure gradient (n, n_out) FP64 of a sorted pressure field."""
        import torch
        out = torch.empty((max(self.n, 1), vct_n_out(self.dim, mask)), dtype=torch.float64, device=self.device)
        vct_grad_sum(self.nl, self.pos, self.vol, self.kernel, self.map_for(mapspec), rho_sorted, rho0, p_sorted, mask,
                     out)
        return out

    def adjoint(self, u_sorted, proj=None, want_dtheta=True):
        """dphi (sorted) and dtheta for the cotangent u of the Laplacian; `proj`
        is the FP64 apply output (1, n, n_out) of the field, needed for dtheta.
        With keep_col the transposed-map form runs, else the push form."""
        import torch
        nt = self.cmap.nterms
        dphi = torch.empty(max(self.n, 1), dtype=torch.float64, device=self.device)
        dth = torch.empty(max(nt, 1), dtype=torch.float64, device=self.device) if want_dtheta else None
        ws = _bytes(lib().vct_adjoint_workspace_size(self.dim, self.n, self.nnz, nt), self.device)
        vct_apply_ops_adjoint(self.nl, self.pos, self.vol, self.kernel, self.state64, self.mask, self.cmap, proj,
                              u_sorted, dphi, dth, ws)
        return dphi[: self.n], (dth[:nt] if dth is not None else None)

    def map_alpha(self, mapspec):
        """J = alpha of the mapping at the sorted particles (n,) FP64."""
        import torch
        out = torch.empty(max(self.n, 1), dtype=torch.float64, device=self.device)
        vct_map_alpha(self.dim, self.n, self.pos, self.map_for(mapspec), out)
        return out[: self.n]

    def jbar_smooth(self, J_sorted, jbar_sorted, cv, re=None):
        """Jbar^N from Jbar^(N-1) (sorted, updated in place) for the Jacobian
        determinants J (sorted); r_e defaults to the support radius."""
        ws = _bytes(lib().vct_jbar_workspace_size(self.n), self.device)
        vct_jbar_smooth(self.nl, self.pos, J_sorted, jbar_sorted, cv, self.R if re is None else re, ws)
        return jbar_sorted

    def adjoint_r2(self, phi_sorted, u_sorted, proj, want_dzhat=False):
        """dtheta (and d loss / d z^, sorted) with physical positions fixed;
        needs a state whose mask holds LAP, PGRAD and PHESS; proj is the FP64
        apply output (1, n, n_out)."""
        import torch
        nt = self.cmap.nterms
        dth = torch.empty(max(nt, 1), dtype=torch.float64, device=self.device)
        dz = torch.empty(max(self.n, 1), dtype=torch.float64, device=self.device) if want_dzhat else None
        ws = _bytes(lib().vct_adjoint_r2_workspace_size(self.dim, self.n, nt), self.device)
        vct_apply_ops_adjoint_r2(self.nl, self.pos, self.vol, self.kernel, self.state64, self.mask, self.cmap, proj,
                                 phi_sorted, u_sorted, dth, dz, ws)
        return dth[:nt], (dz[: self.n] if dz is not None else None)

    def csr_original(self):
        """Neighbour lists in original indices, rows in original order, columns
        ascending (host numpy) -- for comparisons."""
        perm = self.perm[: self.n].cpu().numpy().astype(np.int64)
        rp = self.row_ptr.cpu().numpy()
        col = self.col[: self.nnz].cpu().numpy().astype(np.int64)
        deg = np.diff(rp)
        orig_row = np.repeat(perm, deg)
        orig_col = perm[col]
        order = np.lexsort((orig_col, orig_row))
        new_rp = np.zeros(self.n + 1, dtype=np.int64)
        new_rp[1:] = np.cumsum(np.bincount(orig_row, minlength=self.n))
        return new_rp, orig_col[order]
