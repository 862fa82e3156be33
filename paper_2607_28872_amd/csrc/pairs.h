// Neighbour sums of one field at one particle, shared by the apply and adjoint
// kernels (paper Sec. 3.1, Eqs. gra_1st and sec_SPH2):
//   a_i = sum_j V_j c~_ij phi_ij r~_ij          (d sums)
//   s_i = sum_j V_j F~_ij phi_ij q~_ij          (m sums),
//   F~_ij = c~_ij (r~^T L~_i r~) / |r~|^4,  r~ = r_ij / R.
// A group of G lanes walks the row of particle i with stride G; the caller
// reduces across the group.  T is the arithmetic type of the pair terms and
// sums; the differences r_ij and phi_ij are always formed in FP64 and rounded
// to T once.
#pragma once

#include "common.h"

namespace vct {

template <int D, int KERNEL, class T>
__device__ __forceinline__ void pair_terms(const double* __restrict__ pos, const double* __restrict__ vol,
                                           int64_t n, int64_t j, const double (&xi)[D], double invR,
                                           const T (&L)[Dims<D>::nL], T dphi, T (&acc)[Dims<D>::nk]) {
    using Dm = Dims<D>;
    T r[D];
    T q2 = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        r[a] = T((pos[a * n + j] - xi[a]) * invR);
        q2 += r[a] * r[a];
    }
    T rLr = T(0);
#pragma unroll
    for (int p = 0; p < Dm::nL; ++p)
        rLr += (pair_a<D>(p) == pair_b<D>(p) ? T(1) : T(2)) * L[p] * r[pair_a<D>(p)] * r[pair_b<D>(p)];
    const T c = kernel_shape<KERNEL>(vsqrt(q2));
    const T wa = T(vol[j]) * c * dphi;
    const T ws = wa * rLr * vrcp(q2 * q2);
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] += wa * r[a];
#pragma unroll
    for (int p = 0; p < Dm::m; ++p) acc[D + p] += ws * r[pair_a<D>(p)] * r[pair_b<D>(p)];
}

template <int D, int G, int KERNEL, class T>
__device__ __forceinline__ void row_sums(const double* __restrict__ pos, const double* __restrict__ vol,
                                         const int32_t* __restrict__ col, int64_t n, int64_t rb, int64_t re,
                                         int lane, const double (&xi)[D], double invR, const double* __restrict__ ph,
                                         double phi_i, const T (&L)[Dims<D>::nL], T (&acc)[Dims<D>::nk]) {
#pragma unroll
    for (int c = 0; c < Dims<D>::nk; ++c) acc[c] = T(0);
    for (int64_t k = rb + lane; k < re; k += G) {
        const int64_t j = col[k];
        pair_terms<D, KERNEL, T>(pos, vol, n, j, xi, invR, L, T(ph[j] - phi_i), acc);
    }
#pragma unroll
    for (int c = 0; c < Dims<D>::nk; ++c) acc[c] = group_sum(acc[c], G);
}

}  // namespace vct
