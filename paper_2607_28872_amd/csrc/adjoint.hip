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
#include "pairs.h"

namespace vct {

template <int D, int G, int KERNEL>
__global__ __launch_bounds__(256) void k_adjoint_dphi(int64_t n, const double* __restrict__ pos,
                                                      const double* __restrict__ vol,
                                                      const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, double invR,
                                                      const double* __restrict__ state, int lap_row,
                                                      const double* __restrict__ u, double* __restrict__ dphi) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, nk = Dm::nk, m = Dm::m;
    constexpr int PER_BLOCK = 256 / G;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x % G;
    const int64_t k = (int64_t)tile * PER_BLOCK + threadIdx.x / G;
    if (k >= n) return;
    double xk[D];
#pragma unroll
    for (int a = 0; a < D; ++a) xk[a] = pos[a * n + k];
    double Lk[nL];
#pragma unroll
    for (int p = 0; p < nL; ++p) Lk[p] = state[(int64_t)p * n + k];
    const double* Plap = state + (int64_t)(nL + lap_row * nk) * n;
    const double Vk = vol[k];
    double acc1 = 0.0, acc2[nk];
#pragma unroll
    for (int c = 0; c < nk; ++c) acc2[c] = 0.0;
    const int64_t rb = row_ptr[k], re = row_ptr[k + 1];
    for (int64_t e = rb + lane; e < re; e += G) {
        const int64_t i = col[e];
        double r[D], q2 = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) { r[a] = (pos[a * n + i] - xk[a]) * invR; q2 += r[a] * r[a]; }
        double qv[m];
#pragma unroll
        for (int p = 0; p < m; ++p) qv[p] = r[pair_a<D>(p)] * r[pair_b<D>(p)];
        const double c = kernel_shape<KERNEL>(sqrt(q2));
        const double iq4 = 1.0 / (q2 * q2);
        // k's own row: v_ki with the correction matrix of k
        double rLk = 0.0, rLi = 0.0;
#pragma unroll
        for (int p = 0; p < nL; ++p) {
            const double wgt = (pair_a<D>(p) == pair_b<D>(p) ? 1.0 : 2.0) * qv[p];
            rLk += wgt * Lk[p];
            rLi += wgt * state[(int64_t)p * n + i];
        }
        const double Vi = vol[i];
        const double wa = Vi * c, wsk = Vi * c * rLk * iq4;
#pragma unroll
        for (int a = 0; a < D; ++a) acc2[a] += wa * r[a];
#pragma unroll
        for (int p = 0; p < m; ++p) acc2[D + p] += wsk * qv[p];
        // W_ik from row i: r~_ik = -r~_ki, V_k, correction matrix of i
        const double ca = Vk * c, csi = Vk * c * rLi * iq4;
        double W = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) W -= Plap[(int64_t)a * n + i] * ca * r[a];
#pragma unroll
        for (int p = 0; p < m; ++p) W += Plap[(int64_t)(D + p) * n + i] * csi * qv[p];
        acc1 += u[i] * W;
    }
    acc1 = group_sum(acc1, G);
#pragma unroll
    for (int c = 0; c < nk; ++c) acc2[c] = group_sum(acc2[c], G);
    if (lane == 0) {
        double self = 0.0;
#pragma unroll
        for (int c = 0; c < nk; ++c) self += Plap[(int64_t)c * n + k] * acc2[c];
        dphi[k] = acc1 - u[k] * self;
    }
}

// Per particle: D^ phi from the PGRAD / PHESS rows, then
// xi_k = u_i * d(c_trans . D^)/d h^(k) for the six bottom quantities.
template <int D, int G, int KERNEL>
__global__ __launch_bounds__(256) void k_adjoint_xi(int64_t n, const double* __restrict__ pos,
                                                    const double* __restrict__ vol,
                                                    const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col, double invR,
                                                    const double* __restrict__ state, int pg_row, int ph_row,
                                                    MapParams mp, const double* __restrict__ phi,
                                                    const double* __restrict__ u, double* __restrict__ xi_out) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, nk = Dm::nk;
    constexpr int PER_BLOCK = 256 / G;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x % G;
    const int64_t i = (int64_t)tile * PER_BLOCK + threadIdx.x / G;
    if (i >= n) return;
    double x[D];
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = pos[a * n + i];
    double L[nL];
#pragma unroll
    for (int p = 0; p < nL; ++p) L[p] = state[(int64_t)p * n + i];
    double acc[nk];
    row_sums<D, G, KERNEL, double>(pos, vol, col, n, row_ptr[i], row_ptr[i + 1], lane, x, invR, phi, phi[i], L,
                                   acc);
    // projected derivatives needed by c_trans: dz^, zz, xz, (yz)
    auto row = [&](int o) {
        const double* P = state + (int64_t)(nL + o * nk) * n + i;
        double v = 0.0;
#pragma unroll
        for (int c = 0; c < nk; ++c) v += P[(int64_t)c * n] * acc[c];
        return v;
    };
    const double gz = row(pg_row + D - 1);
    const double Hzz = (D == 3) ? row(ph_row + 2) : row(ph_row + 1);
    const double Hxz = (D == 3) ? row(ph_row + 4) : row(ph_row + 2);
    const double Hyz = (D == 3) ? row(ph_row + 5) : 0.0;
    if (lane != 0) return;
    double h[6];
    bottom6(mp, x[0], D == 3 ? x[1] : 0.0, h);
    Dual6 hd[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        hd[q] = Dual6(h[q]);
        hd[q].d[q] = 1.0;
    }
    const MapCoef<Dual6> mc = map_coef<Dual6>(mp, hd, x[D - 1]);
    const double ui = u[i];
#pragma unroll
    for (int q = 0; q < 6; ++q)
        xi_out[(int64_t)q * n + i] = ui * (mc.c0.d[q] * gz + mc.c3.d[q] * Hzz + mc.c4.d[q] * Hxz + mc.c5.d[q] * Hyz);
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
static int launch_adjoint(int64_t n, const double* pos, const double* vol, const int64_t* row_ptr,
                          const int32_t* col, double invR, const double* state, int lap_row, int pg_row,
                          int ph_row, const MapParams& mp, const double* phi, const double* u, double* dphi,
                          double* dtheta, double* xi, double* partials, hipStream_t s) {
    constexpr int G = (D == 3) ? 8 : 4;
    constexpr int PER_BLOCK = 256 / G;
    const int64_t nb = (n + PER_BLOCK - 1) / PER_BLOCK;
    if (dphi) {
        hipLaunchKernelGGL((k_adjoint_dphi<D, G, KERNEL>), dim3((unsigned)nb), dim3(256), 0, s, n, pos, vol,
                           row_ptr, col, invR, state, lap_row, u, dphi);
        VCT_LAUNCH_CHECK();
    }
    if (dtheta && mp.nterms > 0) {
        hipLaunchKernelGGL((k_adjoint_xi<D, G, KERNEL>), dim3((unsigned)nb), dim3(256), 0, s, n, pos, vol, row_ptr,
                           col, invR, state, pg_row, ph_row, mp, phi, u, xi);
        VCT_LAUNCH_CHECK();
        const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
        hipLaunchKernelGGL(k_dtheta_partials, dim3((unsigned)nred), dim3(kRedThreads), 0, s, n, pos, D, mp, xi,
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
    return aligned_sum({(size_t)n * 6 * sizeof(double), (size_t)(nred > 0 ? nred : 1) * (nterms > 0 ? nterms : 1) * 8});
}

extern "C" int vct_apply_ops_adjoint(int dim, int64_t n, const double* pos_sorted, const double* vol_sorted,
                                     const int64_t* row_ptr, const int32_t* col, int kernel, double R,
                                     const double* state64, uint32_t out_mask, const vct_map* map,
                                     const double* phi_sorted, const double* u, double* dphi, double* dtheta,
                                     void* ws, size_t ws_bytes, void* stream) {
    const uint32_t need = VCT_OUT_LAP | VCT_OUT_PGRAD | VCT_OUT_PHESS;
    if ((dim != 2 && dim != 3) || n < 0 || n > INT32_MAX || !(R > 0.0) || !isfinite(R) || !map ||
        !mask_valid(out_mask) || (out_mask & need) != need ||
        (kernel != VCT_KERNEL_WENDLAND_C2 && kernel != VCT_KERNEL_CUBIC_SPLINE))
        return VCT_E_ARG;
    MapParams mp;
    int st = map_params_from(map, dim, mp);
    if (st) return st;
    hipStream_t s = as_stream(stream);
    if (n == 0) {
        if (dtheta && mp.nterms > 0) {
            hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(64), 0, s, dtheta, (int64_t)mp.nterms);
            VCT_LAUNCH_CHECK();
        }
        return VCT_OK;
    }
    if (!pos_sorted || !vol_sorted || !row_ptr || !col || !state64 || !u) return VCT_E_ARG;
    if (dtheta && !phi_sorted) return VCT_E_ARG;
    if (!ws || ws_bytes < vct_adjoint_workspace_size(dim, n, mp.nterms)) return VCT_E_WORKSPACE;
    Carver cv(ws, ws_bytes);
    double* xi = cv.take<double>((size_t)n * 6);
    const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
    double* partials = cv.take<double>((size_t)nred * (mp.nterms > 0 ? mp.nterms : 1));
    const int lap_row = group_row(dim, out_mask, VCT_OUT_LAP);
    const int pg_row = group_row(dim, out_mask, VCT_OUT_PGRAD);
    const int ph_row = group_row(dim, out_mask, VCT_OUT_PHESS);
    const double invR = 1.0 / R;
    if (dim == 2)
        st = (kernel == VCT_KERNEL_WENDLAND_C2)
                 ? launch_adjoint<2, VCT_KERNEL_WENDLAND_C2>(n, pos_sorted, vol_sorted, row_ptr, col, invR, state64,
                                                             lap_row, pg_row, ph_row, mp, phi_sorted, u, dphi,
                                                             dtheta, xi, partials, s)
                 : launch_adjoint<2, VCT_KERNEL_CUBIC_SPLINE>(n, pos_sorted, vol_sorted, row_ptr, col, invR, state64,
                                                              lap_row, pg_row, ph_row, mp, phi_sorted, u, dphi,
                                                              dtheta, xi, partials, s);
    else
        st = (kernel == VCT_KERNEL_WENDLAND_C2)
                 ? launch_adjoint<3, VCT_KERNEL_WENDLAND_C2>(n, pos_sorted, vol_sorted, row_ptr, col, invR, state64,
                                                             lap_row, pg_row, ph_row, mp, phi_sorted, u, dphi,
                                                             dtheta, xi, partials, s)
                 : launch_adjoint<3, VCT_KERNEL_CUBIC_SPLINE>(n, pos_sorted, vol_sorted, row_ptr, col, invR, state64,
                                                              lap_row, pg_row, ph_row, mp, phi_sorted, u, dphi,
                                                              dtheta, xi, partials, s);
    return st;
}
