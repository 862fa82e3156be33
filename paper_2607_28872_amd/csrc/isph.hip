// Conventional ISPH operators through the vertical coordinate transformation
// (the ISPH case of Table case_names):
//   0th-order models of Sec. 3.1, in the projected space,
//     <grad^ phi>^(0)_i = sum_j V_j phi_ij grad w_ij,
//     <d2 phi / dx^I dx^J>^(0)_i = sum_j V_j (c r^I r^J / |r|^2 - delta^IJ)
//                                  (r_ij . grad w_ij / |r_ij|^2) phi_ij,
//     c = 4 in 2-D and 5 in 3-D (Eq. sec_0th), whose trace is the Brookshaw
//     Laplacian 2 sum_j V_j (r_ij . grad w_ij / |r_ij|^2) phi_ij,
//   mapped to physical space like the SPH(2) derivatives (Eqs. grad_VCT,
//   lap_VCT and the chain rule for the cross terms);
//   summation pressure gradient (Eq. gra_sum), J <grad^ p>^+ with
//     <grad^ p>^+_i = rho_i sum_j m_j (p_j / rho_j^2 + p_i / rho_i^2) grad w_ij,
//     m_j = rho_j V_j.
// For the radial kernels grad w_ij = G(|r_ij|) r_ij with r_ij = r_j - r_i and
// G = -w'(r) / r, so r_ij . grad w_ij / |r_ij|^2 = G.  G is KG c~(q), with
// c~ the kernel shape of the SPH(2) sums and KG the normalisation.
#include <string.h>

#include "common.h"
#include "map_dev.h"
#include "tiles.h"

namespace vct {

int nlist_check(const vct_nlist* nl, Grid& g);

constexpr int kZLanes = 8;                    // lanes per particle
constexpr int kZThreads = kChunk * kZLanes;   // one chunk per work-group
constexpr int kZWin = 1400;                   // LDS window capacity (records)

struct ZeroArgs {
    int64_t n;
    double invR, KG;
    Grid g;
    const double* pos;
    const double* vol;
    const int64_t* row_ptr;
    const uint16_t* col16;
    const int64_t* cs;
    const int32_t* cstart;
    const int4* cinfo;
    const int32_t* cwin;
    const int64_t* nchunks;
    int nf;
    const double* f;      // [nf][n] fields, or the pressure
    const double* rho;    // [n] or NULL (gradient summation)
    double rho0;
    uint32_t mask;
    int nrows;
    double* out;          // [nf][n][nrows]
};

// G / c~: the normalisation of -w'(r)/r (Wendland C2 of unit integral,
// 20 C / R^2; cubic spline with l = R / 2, a_d / l^2)
inline double gfac_norm(int dim, int kernel, double R) {
    if (kernel == VCT_KERNEL_WENDLAND_C2) {
        const double C = dim == 2 ? 7.0 / (M_PI * R * R) : 21.0 / (2.0 * M_PI * R * R * R);
        return 20.0 * C / (R * R);
    }
    const double l = 0.5 * R;
    const double ad = dim == 2 ? 10.0 / (7.0 * M_PI * l * l) : 1.0 / (M_PI * l * l * l);
    return ad / (l * l);
}

// window record of neighbour slot t: position, volume (LDS or global)
template <int D>
__device__ __forceinline__ double4 window_record(const ZeroArgs& A, const WindowT<D>& w, const double4* sd, bool in_lds,
                                                 int t, int64_t& j) {
    if (in_lds) return sd[t];
    j = window_global<D>(w, t);
    const int64_t n = A.n;
    return make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
}

// Per chunk of particles (one work-group, kZLanes lanes per particle), for
// each field: a = sum V c~ phi_ij r~, S_IJ = sum V c~ phi_ij r~_I r~_J / |r~|^2
// and t = sum V c~ phi_ij; then
//   grad^ = KG R a,   H^_IJ = KG (c S_IJ - delta_IJ t)
// and the output rows of the mask at the particle's mapping.
template <int D, int KERNEL>
__global__ __launch_bounds__(kZThreads, 4) void k_ops0(ZeroArgs A, MapParams mp) {
    using Dm = Dims<D>;
    constexpr int m = Dm::m;
    constexpr double cc = D == 2 ? 4.0 : 5.0;
    __shared__ double4 sd[kZWin];
    __shared__ double sf[kZWin];
    __shared__ WindowT<D> w;
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *A.nchunks) return;   // uniform over the work-group
    const int64_t n = A.n;
    const int64_t p0 = A.cstart[b], p1 = A.cstart[b + 1];
    if (threadIdx.x < kWave) {
        if (A.cwin) window_load<D>(A.cwin, b, w);
        else chunk_window_wave<D>(A.g, A.cs, A.cinfo[b], w);
    }
    const int lane = threadIdx.x % kZLanes;
    const int64_t i = p0 + threadIdx.x / kZLanes;
    const bool valid = i < p1;
    const int64_t ii = valid ? i : p0;
    double xi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xi[a] = a < D ? A.pos[a * n + ii] : 0.0;
    __syncthreads();
    const int W = w.off[w.nr];
    const bool in_lds = W <= kZWin;
    if (in_lds) {
        for (int t = threadIdx.x; t < W; t += kZThreads) {
            const int64_t j = window_global<D>(w, t);
            sd[t] = make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
        }
    }
    const int64_t rb = valid ? A.row_ptr[ii] : 0, re = valid ? A.row_ptr[ii + 1] : 0;
    // the mapping at the particle (lane 0 writes)
    const MapCoef<double> mc = map_coef_at(mp, ii, xi[0], D == 3 ? xi[1] : 0.0, xi[D - 1]);
    const bool map_ok = mc.alpha > 0.0 && isfinite(mc.alpha + mc.gx + mc.gy + mc.c0 + mc.zxy);
    const double nanv = __builtin_nan("");
    for (int f = 0; f < A.nf; ++f) {
        const double* F = A.f + (int64_t)f * n;
        if (f > 0) __syncthreads();   // the previous field's reads of sf are done
        if (in_lds)
            for (int t = threadIdx.x; t < W; t += kZThreads) sf[t] = F[window_global<D>(w, t)];
        __syncthreads();
        const double fi = F[ii];
        double acc[D], S[m], ts = 0.0, bad = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) acc[a] = 0.0;
#pragma unroll
        for (int p = 0; p < m; ++p) S[p] = 0.0;
        for (int64_t e = rb + lane; e < re; e += kZLanes) {
            const int t = dcheck((int)A.col16[e], W, kChkWindow);
            int64_t j = 0;
            const double4 q = window_record<D>(A, w, sd, in_lds, t, j);
            const double fj = in_lds ? sf[t] : F[j];
            double r[D];
            r[0] = (q.x - xi[0]) * A.invR;
            r[1] = (q.y - xi[1]) * A.invR;
            if (D == 3) r[D - 1] = (q.z - xi[2]) * A.invR;
            double q2 = r[0] * r[0];
#pragma unroll
            for (int a = 1; a < D; ++a) q2 = fma(r[a], r[a], q2);
            // y = 1/|r~|: |r~| = q2 y, 1/|r~|^2 = y^2; a neighbour at zero (or
            // non-finite) distance makes the particle's outputs NaN
            bad = q2 > 0.0 ? bad : 1.0;
            const double y = vrsq(q2);
            const double fij = q.w * kernel_shape<KERNEL>(q2 * y) * (fj - fi);
            const double u = fij * (y * y);
#pragma unroll
            for (int a = 0; a < D; ++a) acc[a] = fma(fij, r[a], acc[a]);
            ts += fij;
#pragma unroll
            for (int p = 0; p < m; ++p) S[p] = fma(u * r[pair_a<D>(p)], r[pair_b<D>(p)], S[p]);
        }
#pragma unroll
        for (int a = 0; a < D; ++a) acc[a] = group_sum(acc[a], kZLanes);
#pragma unroll
        for (int p = 0; p < m; ++p) S[p] = group_sum(S[p], kZLanes);
        ts = group_sum(ts, kZLanes);
        bad = group_sum(bad, kZLanes);
        if (valid && lane == 0) {
            double pg[D], ph[m];
            const double kr = A.KG / A.invR;
#pragma unroll
            for (int a = 0; a < D; ++a) pg[a] = kr * acc[a];
#pragma unroll
            for (int p = 0; p < m; ++p) ph[p] = A.KG * (p < D ? fma(cc, S[p], -ts) : cc * S[p]);
            double* o = A.out + ((int64_t)f * n + ii) * A.nrows;
            const bool ok = map_ok && bad == 0.0;
            emit_rows<D>(A.mask, mc, pg, ph, [&](int k, double v) { o[k] = ok ? v : nanv; });
        }
    }
}

// Summation gradient of the pressure field f[0]: per particle
// grad^ = rho_i KG R sum_j V_j rho_j (p_j / rho_j^2 + p_i / rho_i^2) c~ r~_ij,
// then J grad^ (GRAD rows) and grad^ (PGRAD rows).
template <int D, int KERNEL>
__global__ __launch_bounds__(kZThreads, 4) void k_grad_sum(ZeroArgs A, MapParams mp) {
    __shared__ double4 sd[kZWin];
    __shared__ double2 sp[kZWin];   // rho_j, p_j / rho_j^2
    __shared__ WindowT<D> w;
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *A.nchunks) return;
    const int64_t n = A.n;
    const int64_t p0 = A.cstart[b], p1 = A.cstart[b + 1];
    if (threadIdx.x < kWave) {
        if (A.cwin) window_load<D>(A.cwin, b, w);
        else chunk_window_wave<D>(A.g, A.cs, A.cinfo[b], w);
    }
    const int lane = threadIdx.x % kZLanes;
    const int64_t i = p0 + threadIdx.x / kZLanes;
    const bool valid = i < p1;
    const int64_t ii = valid ? i : p0;
    double xi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xi[a] = a < D ? A.pos[a * n + ii] : 0.0;
    const double rhoi = A.rho ? A.rho[ii] : A.rho0;
    const double pi_r = A.f[ii] / (rhoi * rhoi);
    __syncthreads();
    const int W = w.off[w.nr];
    const bool in_lds = W <= kZWin;
    if (in_lds) {
        for (int t = threadIdx.x; t < W; t += kZThreads) {
            const int64_t j = window_global<D>(w, t);
            sd[t] = make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
            const double rj = A.rho ? A.rho[j] : A.rho0;
            sp[t] = make_double2(rj, A.f[j] / (rj * rj));
        }
    }
    __syncthreads();
    double acc[D], bad = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] = 0.0;
    const int64_t rb = valid ? A.row_ptr[ii] : 0, re = valid ? A.row_ptr[ii + 1] : 0;
    for (int64_t e = rb + lane; e < re; e += kZLanes) {
        const int t = dcheck((int)A.col16[e], W, kChkWindow);
        int64_t j = 0;
        const double4 q = window_record<D>(A, w, sd, in_lds, t, j);
        double2 pr;
        if (in_lds) {
            pr = sp[t];
        } else {
            const double rj = A.rho ? A.rho[j] : A.rho0;
            pr = make_double2(rj, A.f[j] / (rj * rj));
        }
        double r[D];
        r[0] = (q.x - xi[0]) * A.invR;
        r[1] = (q.y - xi[1]) * A.invR;
        if (D == 3) r[D - 1] = (q.z - xi[2]) * A.invR;
        double q2 = r[0] * r[0];
#pragma unroll
        for (int a = 1; a < D; ++a) q2 = fma(r[a], r[a], q2);
        bad = q2 > 0.0 ? bad : 1.0;
        const double y = vrsq(q2);
        const double s = q.w * pr.x * (pr.y + pi_r) * kernel_shape<KERNEL>(q2 * y);
#pragma unroll
        for (int a = 0; a < D; ++a) acc[a] = fma(s, r[a], acc[a]);
    }
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] = group_sum(acc[a], kZLanes);
    bad = group_sum(bad, kZLanes);
    if (!valid || lane != 0) return;
    const MapCoef<double> mc = map_coef_at(mp, ii, xi[0], D == 3 ? xi[1] : 0.0, xi[D - 1]);
    const bool map_ok = mc.alpha > 0.0 && isfinite(mc.alpha + mc.gx + mc.gy) && bad == 0.0;
    const double nanv = __builtin_nan("");
    double pg[D], ph[Dims<D>::m];
    const double kr = rhoi * A.KG / A.invR;
#pragma unroll
    for (int a = 0; a < D; ++a) pg[a] = kr * acc[a];
#pragma unroll
    for (int p = 0; p < Dims<D>::m; ++p) ph[p] = 0.0;
    double* o = A.out + ii * A.nrows;
    emit_rows<D>(A.mask, mc, pg, ph, [&](int k, double v) { o[k] = map_ok ? v : nanv; });
}

static int zero_common(const vct_nlist* nl, Grid& g, const double* pos_sorted, const double* vol_sorted, int kernel,
                       const vct_map* map, uint32_t mask, uint32_t allowed, ZeroArgs& a, MapParams& mp) {
    int st = nlist_check(nl, g);
    if (st) return st;
    if (!map || !mask || (mask & ~allowed) || (kernel != VCT_KERNEL_WENDLAND_C2 && kernel != VCT_KERNEL_CUBIC_SPLINE))
        return VCT_E_ARG;
    st = map_params_from(map, nl->dim, nl->n, mp);
    if (st) return st;
    const int64_t n = nl->n;
    if (n > 0 && (!pos_sorted || !vol_sorted || !nl->col16)) return VCT_E_ARG;
    const int64_t ncols = nl->dim == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    memset(&a, 0, sizeof(a));
    a.n = n; a.invR = 1.0 / nl->R; a.KG = gfac_norm(nl->dim, kernel, nl->R); a.g = g;
    a.pos = pos_sorted; a.vol = vol_sorted;
    a.row_ptr = nl->row_ptr; a.col16 = nl->col16; a.cs = nl->cell_start; a.cstart = nl->chunk_start;
    a.cinfo = reinterpret_cast<const int4*>(nl->chunk_info); a.cwin = nl->chunk_win;
    a.nchunks = nl->chunk_off + ncols;
    a.mask = mask; a.nrows = n_out_rows(nl->dim, mask);
    return VCT_OK;
}

static int64_t zero_cap(const vct_nlist* nl, const Grid& g) {
    const int64_t ncols = nl->dim == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    return ncols + nl->n / kChunk + 1;
}

VCT_CHECKS_TU(checks_isph)

}  // namespace vct

using namespace vct;

extern "C" int vct_apply_ops0(const vct_nlist* nl, int nf, const double* phi_sorted, const double* pos_sorted,
                              const double* vol_sorted, int kernel, const vct_map* map, uint32_t out_mask, double* out,
                              void* stream) {
    VCT_API_RANGE("vct_apply_ops0");
    Grid g;
    ZeroArgs a;
    MapParams mp;
    const uint32_t allowed = VCT_OUT_GRAD | VCT_OUT_LAP | VCT_OUT_CROSS | VCT_OUT_HESS | VCT_OUT_PGRAD |
                             VCT_OUT_PHESS | VCT_OUT_PZ;
    int st = zero_common(nl, g, pos_sorted, vol_sorted, kernel, map, out_mask, allowed, a, mp);
    if (st) return st;
    if (nf < 0) return VCT_E_ARG;
    if (nl->n == 0 || nf == 0) return VCT_OK;
    if (!phi_sorted || !out) return VCT_E_ARG;
    a.nf = nf; a.f = phi_sorted; a.out = out;
    hipStream_t s = as_stream(stream);
    const int64_t cap = zero_cap(nl, g);
#define VCT_OPS0(D, K) VCT_LAUNCH("k_ops0", (k_ops0<D, K>), dim3((unsigned)cap), dim3(kZThreads), 0, s, a, mp)
    if (nl->dim == 2) {
        if (kernel == VCT_KERNEL_WENDLAND_C2) VCT_OPS0(2, VCT_KERNEL_WENDLAND_C2);
        else VCT_OPS0(2, VCT_KERNEL_CUBIC_SPLINE);
    } else {
        if (kernel == VCT_KERNEL_WENDLAND_C2) VCT_OPS0(3, VCT_KERNEL_WENDLAND_C2);
        else VCT_OPS0(3, VCT_KERNEL_CUBIC_SPLINE);
    }
#undef VCT_OPS0
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

extern "C" int vct_grad_sum(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                            const vct_map* map, const double* rho, double rho0, const double* p, uint32_t out_mask,
                            double* out, void* stream) {
    VCT_API_RANGE("vct_grad_sum");
    Grid g;
    ZeroArgs a;
    MapParams mp;
    int st = zero_common(nl, g, pos_sorted, vol_sorted, kernel, map, out_mask, VCT_OUT_GRAD | VCT_OUT_PGRAD, a, mp);
    if (st) return st;
    if (!rho && !(rho0 != 0.0 && isfinite(rho0))) return VCT_E_ARG;
    if (nl->n == 0) return VCT_OK;
    if (!p || !out) return VCT_E_ARG;
    a.nf = 1; a.f = p; a.rho = rho; a.rho0 = rho0; a.out = out;
    hipStream_t s = as_stream(stream);
    const int64_t cap = zero_cap(nl, g);
#define VCT_GSUM(D, K) VCT_LAUNCH("k_grad_sum", (k_grad_sum<D, K>), dim3((unsigned)cap), dim3(kZThreads), 0, s, a, mp)
    if (nl->dim == 2) {
        if (kernel == VCT_KERNEL_WENDLAND_C2) VCT_GSUM(2, VCT_KERNEL_WENDLAND_C2);
        else VCT_GSUM(2, VCT_KERNEL_CUBIC_SPLINE);
    } else {
        if (kernel == VCT_KERNEL_WENDLAND_C2) VCT_GSUM(3, VCT_KERNEL_WENDLAND_C2);
        else VCT_GSUM(3, VCT_KERNEL_CUBIC_SPLINE);
    }
#undef VCT_GSUM
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}
