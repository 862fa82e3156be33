// Adjoint of the physical Laplacian operator (built on paper Eqs. lap_VCT and
// sec_SPH2; the adjoint itself is not in the paper).
//
// With lap_i = sum_{j in S_i} W_ij (phi_j - phi_i) and W_ij = P_lap,i . v_ij,
// v_ij = [V_j c~ r~_ij ; V_j F~_ij q~_ij] (F~_ij uses the correction matrix of
// particle i), the field cotangent is
//   dphi_k = sum_{i in S_k} u_i W_ik  -  u_k P_lap,k . sum_{j in S_k} v_kj .
// The neighbour relation is symmetric (the test |r_ij| < R is), so both terms
// are gathers over the row of k: no atomics and a fixed summation order.
//
// Bathymetry coefficients enter only through the VCT coefficients (projected
// positions are held fixed), so
//   dtheta_t = sum_i u_i (d c_trans_i / d coef_t) . D^ phi_i ,
// with d c_trans / d (h, h_x, h_y, h_xx, h_xy, h_yy) from forward-mode dual
// numbers and d h^(k) / d coef_t the t-th term's basis products.  Per-particle
// contributions are reduced per work-group, then across work-groups, in a
// fixed order.
#include "common.h"
#include "map_dev.h"
#include "tiles.h"

namespace vct {

int nlist_check(const vct_nlist* nl, Grid& g);

constexpr int kALanes = 4;                     // lanes per particle
constexpr int kAThreads = kChunk * kALanes;    // one chunk per work-group
constexpr int kAWin = 1280;                    // LDS window capacity (records)
constexpr int kCoef = 16;                      // packed per-particle adjoint record

// Per particle: [L~ (nL), P_lap (d + m), u], one 128-byte record, so the
// gather of a neighbour's coefficients touches a single cache line.
template <int D>
__global__ void k_adjoint_pack(int64_t n, const double* __restrict__ state, int lap_row,
                               const double* __restrict__ u, double* __restrict__ coef) {
    using Dm = Dims<D>;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double* c = coef + i * kCoef;
#pragma unroll
    for (int p = 0; p < Dm::nL; ++p) c[p] = state[(int64_t)p * n + i];
#pragma unroll
    for (int k = 0; k < Dm::nk; ++k) c[Dm::nL + k] = state[(int64_t)(Dm::nL + lap_row * Dm::nk + k) * n + i];
    c[Dm::nL + Dm::nk] = u[i];
}

struct AdjArgs {
    int64_t n;
    double invR;
    Grid g;
    const double* pos;
    const double* vol;
    const double* phi;
    const double* state;
    const double* u;
    const double* coef;
    const int64_t* row_ptr;
    const uint16_t* col16;
    const int64_t* cs;
    const int32_t* cstart;
    const int4* cinfo;
    const int64_t* nchunks;
    int pg_row, ph_row;
    double* dphi;
    double* xi;
};

template <int D, int KERNEL>
__global__ __launch_bounds__(kAThreads) void k_adjoint_dphi(AdjArgs A) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, nk = Dm::nk, m = Dm::m;
    __shared__ double sx[D][kAWin];
    __shared__ double sv[kAWin];
    __shared__ int32_t sj[kAWin];
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *A.nchunks) return;
    const int64_t n = A.n;
    const int64_t p0 = A.cstart[b], p1 = A.cstart[b + 1];
    __shared__ WindowT<D> w;   // one copy per work-group: runtime-indexed, so kept in LDS
    if (threadIdx.x == 0) chunk_window<D>(A.g, A.cs, A.cinfo[b], w);
    __syncthreads();
    const int W = w.off[w.nr];
    const bool in_lds = W <= kAWin;
    if (in_lds) {
        for (int t = threadIdx.x; t < W; t += kAThreads) {
            const int64_t j = window_global<D>(w, t);
#pragma unroll
            for (int a = 0; a < D; ++a) sx[a][t] = A.pos[a * n + j];
            sv[t] = A.vol[j];
            sj[t] = (int32_t)j;
        }
    }
    __syncthreads();
    const int lane = threadIdx.x % kALanes;
    const int64_t k = p0 + threadIdx.x / kALanes;
    if (k >= p1) return;   // whole groups leave together; no barrier follows
    double xk[D];
#pragma unroll
    for (int a = 0; a < D; ++a) xk[a] = A.pos[a * n + k];
    const double* ck = A.coef + k * kCoef;
    double Lk2[nL];
#pragma unroll
    for (int p = 0; p < nL; ++p) Lk2[p] = (pair_a<D>(p) == pair_b<D>(p) ? 1.0 : 2.0) * ck[p];
    const double Vk = A.vol[k];
    double acc1 = 0.0, acc2[nk];
#pragma unroll
    for (int c = 0; c < nk; ++c) acc2[c] = 0.0;
    const int64_t rb = A.row_ptr[k], re = A.row_ptr[k + 1];
    for (int64_t e = rb + lane; e < re; e += kALanes) {
        const int t = A.col16[e];
        double r[D], q2 = 0.0, Vi;
        int64_t i;
        if (in_lds) {
#pragma unroll
            for (int a = 0; a < D; ++a) r[a] = (sx[a][t] - xk[a]) * A.invR;
            Vi = sv[t];
            i = sj[t];
        } else {
            i = window_global<D>(w, t);
#pragma unroll
            for (int a = 0; a < D; ++a) r[a] = (A.pos[a * n + i] - xk[a]) * A.invR;
            Vi = A.vol[i];
        }
#pragma unroll
        for (int a = 0; a < D; ++a) q2 += r[a] * r[a];
        double qv[m];
#pragma unroll
        for (int p = 0; p < m; ++p) qv[p] = r[pair_a<D>(p)] * r[pair_b<D>(p)];
        const double c = kernel_shape<KERNEL>(sqrt(q2));
        const double iq4 = 1.0 / (q2 * q2);
        const double* ci = A.coef + i * kCoef;
        double rLk = 0.0, rLi = 0.0;
#pragma unroll
        for (int p = 0; p < nL; ++p) {
            rLk += Lk2[p] * qv[p];
            rLi += (pair_a<D>(p) == pair_b<D>(p) ? 1.0 : 2.0) * ci[p] * qv[p];
        }
        // k's own row: v_ki with the correction matrix of k
        const double wa = Vi * c, wsk = Vi * c * rLk * iq4;
#pragma unroll
        for (int a = 0; a < D; ++a) acc2[a] += wa * r[a];
#pragma unroll
        for (int p = 0; p < m; ++p) acc2[D + p] += wsk * qv[p];
        // W_ik from row i: r~_ik = -r~_ki, volume V_k, correction matrix of i
        const double ca = Vk * c, csi = Vk * c * rLi * iq4;
        double Wik = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) Wik -= ci[nL + a] * ca * r[a];
#pragma unroll
        for (int p = 0; p < m; ++p) Wik += ci[nL + D + p] * csi * qv[p];
        acc1 += ci[nL + nk] * Wik;
    }
    acc1 = group_sum(acc1, kALanes);
#pragma unroll
    for (int c = 0; c < nk; ++c) acc2[c] = group_sum(acc2[c], kALanes);
    if (lane == 0) {
        double self = 0.0;
#pragma unroll
        for (int c = 0; c < nk; ++c) self += ck[nL + c] * acc2[c];
        A.dphi[k] = acc1 - ck[nL + nk] * self;
    }
}

// Per particle: D^ phi from the PGRAD / PHESS rows, then
// xi_k = u_i * d(c_trans . D^)/d h^(k) for the six bottom quantities.
template <int D, int KERNEL>
__global__ __launch_bounds__(kAThreads) void k_adjoint_xi(AdjArgs A, MapParams mp) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, nk = Dm::nk, m = Dm::m;
    __shared__ double sx[D][kAWin];
    __shared__ double sv[kAWin];
    __shared__ double sp[kAWin];
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *A.nchunks) return;
    const int64_t n = A.n;
    const int64_t p0 = A.cstart[b], p1 = A.cstart[b + 1];
    __shared__ WindowT<D> w;   // one copy per work-group: runtime-indexed, so kept in LDS
    if (threadIdx.x == 0) chunk_window<D>(A.g, A.cs, A.cinfo[b], w);
    __syncthreads();
    const int W = w.off[w.nr];
    const bool in_lds = W <= kAWin;
    if (in_lds) {
        for (int t = threadIdx.x; t < W; t += kAThreads) {
            const int64_t j = window_global<D>(w, t);
#pragma unroll
            for (int a = 0; a < D; ++a) sx[a][t] = A.pos[a * n + j];
            sv[t] = A.vol[j];
            sp[t] = A.phi[j];
        }
    }
    __syncthreads();
    const int lane = threadIdx.x % kALanes;
    const int64_t i = p0 + threadIdx.x / kALanes;
    if (i >= p1) return;   // whole groups leave together; no barrier follows
    double x[D];
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = A.pos[a * n + i];
    double L2[nL];
#pragma unroll
    for (int p = 0; p < nL; ++p) L2[p] = (pair_a<D>(p) == pair_b<D>(p) ? 1.0 : 2.0) * A.state[(int64_t)p * n + i];
    const double phi_i = A.phi[i];
    double acc[nk];
#pragma unroll
    for (int c = 0; c < nk; ++c) acc[c] = 0.0;
    const int64_t rb = A.row_ptr[i], re = A.row_ptr[i + 1];
    for (int64_t e = rb + lane; e < re; e += kALanes) {
        const int t = A.col16[e];
        double r[D], q2 = 0.0, V, pj;
        if (in_lds) {
#pragma unroll
            for (int a = 0; a < D; ++a) r[a] = (sx[a][t] - x[a]) * A.invR;
            V = sv[t];
            pj = sp[t];
        } else {
            const int64_t j = window_global<D>(w, t);
#pragma unroll
            for (int a = 0; a < D; ++a) r[a] = (A.pos[a * n + j] - x[a]) * A.invR;
            V = A.vol[j];
            pj = A.phi[j];
        }
#pragma unroll
        for (int a = 0; a < D; ++a) q2 += r[a] * r[a];
        double qv[m];
#pragma unroll
        for (int p = 0; p < m; ++p) qv[p] = r[pair_a<D>(p)] * r[pair_b<D>(p)];
        double rLr = 0.0;
#pragma unroll
        for (int p = 0; p < nL; ++p) rLr += L2[p] * qv[p];
        const double wa = V * kernel_shape<KERNEL>(sqrt(q2)) * (pj - phi_i);
        const double ws = wa * rLr / (q2 * q2);
#pragma unroll
        for (int a = 0; a < D; ++a) acc[a] += wa * r[a];
#pragma unroll
        for (int p = 0; p < m; ++p) acc[D + p] += ws * qv[p];
    }
#pragma unroll
    for (int c = 0; c < nk; ++c) acc[c] = group_sum(acc[c], kALanes);
    if (lane != 0) return;
    auto row = [&](int o) {
        const double* P = A.state + (int64_t)(nL + o * nk) * n + i;
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < nk; ++c) v += P[(int64_t)c * n] * acc[c];
        return v;
    };
    // projected derivatives needed by c_trans: dz^, zz, xz, (yz)
    const double gz = row(A.pg_row + D - 1);
    const double Hzz = (D == 3) ? row(A.ph_row + 2) : row(A.ph_row + 1);
    const double Hxz = (D == 3) ? row(A.ph_row + 4) : row(A.ph_row + 2);
    const double Hyz = (D == 3) ? row(A.ph_row + 5) : 0.0;
    double h[6];
    bottom6(mp, x[0], D == 3 ? x[1] : 0.0, h);
    Dual6 hd[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        hd[q] = Dual6(h[q]);
        hd[q].d[q] = 1.0;
    }
    const MapCoef<Dual6> mc = map_coef<Dual6>(mp, hd, x[D - 1]);
    const double ui = A.u[i];
#pragma unroll
    for (int q = 0; q < 6; ++q)
        A.xi[(int64_t)q * n + i] = ui * (mc.c0.d[q] * gz + mc.c3.d[q] * Hzz + mc.c4.d[q] * Hxz + mc.c5.d[q] * Hyz);
}

constexpr int kRedThreads = 256;

__global__ __launch_bounds__(kRedThreads) void k_dtheta_partials(int64_t n, const double* __restrict__ pos,
                                                                  int dim, MapParams mp,
                                                                  const double* __restrict__ xi,
                                                                  double* __restrict__ partials) {
    __shared__ double red[kRedThreads];
    const int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x;
    double xv[6] = {0, 0, 0, 0, 0, 0};
    double x = 0.0, y = 0.0;
    if (i < n) {
        for (int q = 0; q < 6; ++q) xv[q] = xi[(int64_t)q * n + i];
        x = pos[i];
        y = (dim == 3) ? pos[n + i] : 0.0;
    }
    for (int t = 0; t < mp.nterms; ++t) {
        double v = 0.0;
        if (i < n) {
            double o[6];
            term_derivs(mp, t, x, y, o);
            for (int q = 0; q < 6; ++q) v += xv[q] * o[q];
        }
        red[threadIdx.x] = v;
        __syncthreads();
        for (int s = kRedThreads / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * mp.nterms + t] = red[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(kRedThreads) void k_dtheta_final(int64_t nblocks, int nterms,
                                                              const double* __restrict__ partials,
                                                              double* __restrict__ dtheta) {
    __shared__ double red[kRedThreads];
    const int t = blockIdx.x;
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < nblocks; b += kRedThreads) v += partials[b * nterms + t];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) dtheta[t] = red[0];
}

template <int D, int KERNEL>
static int launch_adjoint(AdjArgs a, int64_t cap, const MapParams& mp, int lap_row, double* dtheta,
                          double* partials, hipStream_t s) {
    const int64_t n = a.n;
    if (a.dphi) {
        hipLaunchKernelGGL((k_adjoint_pack<D>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, a.state,
                           lap_row, a.u, const_cast<double*>(a.coef));
        VCT_LAUNCH_CHECK();
        hipLaunchKernelGGL((k_adjoint_dphi<D, KERNEL>), dim3((unsigned)cap), dim3(kAThreads), 0, s, a);
        VCT_LAUNCH_CHECK();
    }
    if (dtheta && mp.nterms > 0) {
        hipLaunchKernelGGL((k_adjoint_xi<D, KERNEL>), dim3((unsigned)cap), dim3(kAThreads), 0, s, a, mp);
        VCT_LAUNCH_CHECK();
        const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
        hipLaunchKernelGGL(k_dtheta_partials, dim3((unsigned)nred), dim3(kRedThreads), 0, s, n, a.pos, D, mp, a.xi,
                           partials);
        VCT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_dtheta_final, dim3((unsigned)mp.nterms), dim3(kRedThreads), 0, s, nred, mp.nterms,
                           partials, dtheta);
        VCT_LAUNCH_CHECK();
    }
    return VCT_OK;
}

__global__ void k_zero_f64(double* p, int64_t cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = 0.0;
}

}  // namespace vct

using namespace vct;

extern "C" size_t vct_adjoint_workspace_size(int dim, int64_t n, int nterms) {
    if ((dim != 2 && dim != 3) || n < 0 || nterms < 0) return 0;
    const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
    return aligned_sum({(size_t)n * 6 * sizeof(double), (size_t)(nred > 0 ? nred : 1) * (nterms > 0 ? nterms : 1) * 8,
                        (size_t)n * kCoef * sizeof(double)});
}

extern "C" int vct_apply_ops_adjoint(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted,
                                     int kernel, const double* state64, uint32_t out_mask, const vct_map* map,
                                     const double* phi_sorted, const double* u, double* dphi, double* dtheta,
                                     void* ws, size_t ws_bytes, void* stream) {
    const uint32_t need = VCT_OUT_LAP | VCT_OUT_PGRAD | VCT_OUT_PHESS;
    Grid g;
    int st = nlist_check(nl, g);
    if (st) return st;
    const int dim = nl->dim;
    const int64_t n = nl->n;
    if (!map || !mask_valid(out_mask) || (out_mask & need) != need ||
        (kernel != VCT_KERNEL_WENDLAND_C2 && kernel != VCT_KERNEL_CUBIC_SPLINE))
        return VCT_E_ARG;
    MapParams mp;
    st = map_params_from(map, dim, mp);
    if (st) return st;
    hipStream_t s = as_stream(stream);
    if (n == 0) {
        if (dtheta && mp.nterms > 0) {
            hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, dtheta, (int64_t)mp.nterms);
            VCT_LAUNCH_CHECK();
        }
        return VCT_OK;
    }
    if (!pos_sorted || !vol_sorted || !nl->col16 || !state64 || !u) return VCT_E_ARG;
    if (dtheta && !phi_sorted) return VCT_E_ARG;
    if (!ws || ws_bytes < vct_adjoint_workspace_size(dim, n, mp.nterms)) return VCT_E_WORKSPACE;
    Carver cv(ws, ws_bytes);
    double* xi = cv.take<double>((size_t)n * 6);
    const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
    double* partials = cv.take<double>((size_t)nred * (mp.nterms > 0 ? mp.nterms : 1));
    double* coef = cv.take<double>((size_t)n * kCoef);
    const int64_t ncols = dim == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    AdjArgs a;
    a.n = n; a.invR = 1.0 / nl->R; a.g = g; a.pos = pos_sorted; a.vol = vol_sorted; a.phi = phi_sorted;
    a.state = state64; a.u = u; a.coef = coef; a.row_ptr = nl->row_ptr; a.col16 = nl->col16; a.cs = nl->cell_start;
    a.cstart = nl->chunk_start; a.cinfo = reinterpret_cast<const int4*>(nl->chunk_info);
    a.nchunks = nl->chunk_off + ncols;
    a.pg_row = group_row(dim, out_mask, VCT_OUT_PGRAD);
    a.ph_row = group_row(dim, out_mask, VCT_OUT_PHESS);
    a.dphi = dphi; a.xi = xi;
    const int lap_row = group_row(dim, out_mask, VCT_OUT_LAP);
    const int64_t cap = ncols + n / kChunk + 1;
    if (dim == 2)
        st = (kernel == VCT_KERNEL_WENDLAND_C2)
                 ? launch_adjoint<2, VCT_KERNEL_WENDLAND_C2>(a, cap, mp, lap_row, dtheta, partials, s)
                 : launch_adjoint<2, VCT_KERNEL_CUBIC_SPLINE>(a, cap, mp, lap_row, dtheta, partials, s);
    else
        st = (kernel == VCT_KERNEL_WENDLAND_C2)
                 ? launch_adjoint<3, VCT_KERNEL_WENDLAND_C2>(a, cap, mp, lap_row, dtheta, partials, s)
                 : launch_adjoint<3, VCT_KERNEL_CUBIC_SPLINE>(a, cap, mp, lap_row, dtheta, partials, s);
    return st;
}
