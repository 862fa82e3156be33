// Operator application (paper Sec. 3.1, Eqs. gra_1st and sec_SPH2; Sec. 2.1,
// Eqs. grad_VCT and lap_VCT): the neighbour sums [a_i; s_i] of each field,
// then out_i = P_i [a_i; s_i] with the per-particle state of vct_moments.
//
// Numerics.  phi_ij is dominated by its first-order part r_ij . grad phi,
// which cancels across a (nearly) symmetric neighbourhood in s_i; rounding the
// individual terms is then amplified by |grad phi| / (R |Hess phi|).  The
// kernel therefore sums in two passes: pass 1 forms the first-order gradient
// G = L a (only d sums), pass 2 sums the residual psi_ij = phi_ij - r_ij . G,
// formed in FP64 and second-order small, and the output adds back W G, the
// exact response of the operator to the linear field r . G.  The result is the
// same linear operator; only the rounding changes.
//
// One group of G lanes per particle walks its CSR row (coalesced column reads,
// neighbours of consecutive cell-sorted particles shared in L1/L2), the group
// reduces its sums with cross-lane shuffles, and lane o of the group produces
// output row o.  Work-groups are remapped so each XCD covers a contiguous
// range of particles; the second pass re-reads the row from cache.
#include "common.h"
#include "pairs.h"

namespace vct {

template <int D, int G, int KERNEL, class T, class S>
__global__ __launch_bounds__(256) void k_apply(int64_t n, int nf, const double* __restrict__ phi,
                                               const double* __restrict__ pos, const double* __restrict__ vol,
                                               const int64_t* __restrict__ row_ptr,
                                               const int32_t* __restrict__ col, double invR,
                                               const S* __restrict__ state, int nrows,
                                               double* __restrict__ out) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, nk = Dm::nk;
    constexpr int PER_BLOCK = 256 / G;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x % G;
    const int64_t i = (int64_t)tile * PER_BLOCK + threadIdx.x / G;
    if (i >= n) return;
    double xi[D];
#pragma unroll
    for (int a = 0; a < D; ++a) xi[a] = pos[a * n + i];
    T L[nL];
#pragma unroll
    for (int p = 0; p < nL; ++p) L[p] = T(state[(int64_t)p * n + i]);
    const int64_t rb = row_ptr[i], re = row_ptr[i + 1];
    const S* Wst = state + (int64_t)(nL + nrows * nk) * n + i;
    for (int f = 0; f < nf; ++f) {
        const double* ph = phi + (int64_t)f * n;
        const double phi_i = ph[i];
        // pass 1: first-order sums a_i and the gradient G~ = L~ a~ (units of 1/R)
        T a1[D];
#pragma unroll
        for (int a = 0; a < D; ++a) a1[a] = T(0);
        for (int64_t k = rb + lane; k < re; k += G) {
            const int64_t j = col[k];
            T r[D], q2 = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                r[a] = T((pos[a * n + j] - xi[a]) * invR);
                q2 += r[a] * r[a];
            }
            const T w = T(vol[j]) * kernel_shape<KERNEL>(vsqrt(q2)) * T(ph[j] - phi_i);
#pragma unroll
            for (int a = 0; a < D; ++a) a1[a] += w * r[a];
        }
#pragma unroll
        for (int a = 0; a < D; ++a) a1[a] = group_sum(a1[a], G);
        double Gt[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            T t = T(0);
#pragma unroll
            for (int b = 0; b < D; ++b) t += L[sym_index<D>(a, b)] * a1[b];
            Gt[a] = (double)t;
        }
        // pass 2: sums of the residual psi_ij = phi_ij - r~_ij . G~ (formed in FP64)
        T acc[nk];
#pragma unroll
        for (int c = 0; c < nk; ++c) acc[c] = T(0);
        for (int64_t k = rb + lane; k < re; k += G) {
            const int64_t j = col[k];
            double psi = ph[j] - phi_i;
#pragma unroll
            for (int a = 0; a < D; ++a) psi -= (pos[a * n + j] - xi[a]) * invR * Gt[a];
            pair_terms<D, KERNEL, T>(pos, vol, n, j, xi, invR, L, T(psi), acc);
        }
#pragma unroll
        for (int c = 0; c < nk; ++c) acc[c] = group_sum(acc[c], G);
        for (int o = lane; o < nrows; o += G) {
            const S* P = state + (int64_t)(nL + o * nk) * n + i;
            T v = T(0);
#pragma unroll
            for (int c = 0; c < nk; ++c) v += T(P[(int64_t)c * n]) * acc[c];
            T lin = T(0);
#pragma unroll
            for (int a = 0; a < D; ++a) lin += T(Wst[(int64_t)(o * D + a) * n]) * T(Gt[a]);
            out[((int64_t)f * n + i) * nrows + o] = (double)v + (double)lin * invR;
        }
    }
}

template <int D, int KERNEL, class T, class S>
static int launch_apply(int64_t n, int nf, const double* phi, const double* pos, const double* vol,
                        const int64_t* row_ptr, const int32_t* col, double invR, const S* state, int nrows,
                        double* out, hipStream_t s) {
    constexpr int G = (D == 3) ? 8 : 4;
    constexpr int PER_BLOCK = 256 / G;
    int64_t nb = (n + PER_BLOCK - 1) / PER_BLOCK;
    hipLaunchKernelGGL((k_apply<D, G, KERNEL, T, S>), dim3((unsigned)nb), dim3(256), 0, s, n, nf, phi, pos, vol,
                       row_ptr, col, invR, state, nrows, out);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

template <int D, class T, class S>
static int dispatch_kernel(int kernel, int64_t n, int nf, const double* phi, const double* pos, const double* vol,
                           const int64_t* row_ptr, const int32_t* col, double invR, const S* state, int nrows,
                           double* out, hipStream_t s) {
    if (kernel == VCT_KERNEL_WENDLAND_C2)
        return launch_apply<D, VCT_KERNEL_WENDLAND_C2, T, S>(n, nf, phi, pos, vol, row_ptr, col, invR, state,
                                                             nrows, out, s);
    return launch_apply<D, VCT_KERNEL_CUBIC_SPLINE, T, S>(n, nf, phi, pos, vol, row_ptr, col, invR, state, nrows,
                                                          out, s);
}

template <class T, class S>
static int dispatch_dim(int dim, int kernel, int64_t n, int nf, const double* phi, const double* pos,
                        const double* vol, const int64_t* row_ptr, const int32_t* col, double invR, const S* state,
                        int nrows, double* out, hipStream_t s) {
    if (dim == 2)
        return dispatch_kernel<2, T, S>(kernel, n, nf, phi, pos, vol, row_ptr, col, invR, state, nrows, out, s);
    return dispatch_kernel<3, T, S>(kernel, n, nf, phi, pos, vol, row_ptr, col, invR, state, nrows, out, s);
}

}  // namespace vct

using namespace vct;

extern "C" int vct_apply_ops(int dim, int64_t n, int nf, const double* phi_sorted, const double* pos_sorted,
                             const double* vol_sorted, const int64_t* row_ptr, const int32_t* col, int kernel,
                             double R, const void* state, uint32_t out_mask, int precision, double* out,
                             void* stream) {
    if ((dim != 2 && dim != 3) || n < 0 || n > INT32_MAX || nf < 1 || !(R > 0.0) || !isfinite(R) ||
        !mask_valid(out_mask) || (kernel != VCT_KERNEL_WENDLAND_C2 && kernel != VCT_KERNEL_CUBIC_SPLINE) ||
        (precision != VCT_FP64 && precision != VCT_MIXED && precision != VCT_MIXED_S64))
        return VCT_E_ARG;
    if (n == 0) return VCT_OK;
    if (!phi_sorted || !pos_sorted || !vol_sorted || !row_ptr || !col || !state || !out) return VCT_E_ARG;
    const int nrows = n_out_rows(dim, out_mask);
    const double invR = 1.0 / R;
    hipStream_t s = as_stream(stream);
    switch (precision) {
    case VCT_FP64:
        return dispatch_dim<double, double>(dim, kernel, n, nf, phi_sorted, pos_sorted, vol_sorted, row_ptr, col,
                                            invR, static_cast<const double*>(state), nrows, out, s);
    case VCT_MIXED:
        return dispatch_dim<float, float>(dim, kernel, n, nf, phi_sorted, pos_sorted, vol_sorted, row_ptr, col,
                                          invR, static_cast<const float*>(state), nrows, out, s);
    default:
        return dispatch_dim<float, double>(dim, kernel, n, nf, phi_sorted, pos_sorted, vol_sorted, row_ptr, col,
                                           invR, static_cast<const double*>(state), nrows, out, s);
    }
}
