// Weight of one neighbour in the physical Laplacian (Eqs. lap_VCT and
// sec_SPH2): lap_i = sum_{j in S_i} W_ij (phi_j - phi_i) with
//   W_ij = V_j c~_ij [P_a,i . r~_ij + (r~_ij' L~_i r~_ij) / |r~_ij|^4 P_s,i . q~_ij],
// r~ = r / R, c~ the kernel shape, L~_i particle i's first-order correction
// matrix (L2: upper triangle, off-diagonals doubled) and P_a,i, P_s,i the
// first- and second-order parts of its Laplacian row of the state (Pl, any
// common factor folded in).  Shared by the adjoint and the pressure solver.
#pragma once

#include "common.h"

namespace vct {

template <int D, int KERNEL>
__device__ __forceinline__ double lap_weight(const double4& q, const double (&xi)[3], double invR,
                                             const double (&L2)[Dims<D>::nL], const double (&Pl)[Dims<D>::nk]) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, m = Dm::m;
    double r[D];
    r[0] = (q.x - xi[0]) * invR;
    r[1] = (q.y - xi[1]) * invR;
    if (D == 3) r[D - 1] = (q.z - xi[2]) * invR;
    double q2 = r[0] * r[0];
#pragma unroll
    for (int a = 1; a < D; ++a) q2 = fma(r[a], r[a], q2);
    double qv[m];
#pragma unroll
    for (int p = 0; p < m; ++p) qv[p] = r[pair_a<D>(p)] * r[pair_b<D>(p)];
    double rLr = L2[0] * qv[0], sa = Pl[0] * r[0], ss = Pl[D] * qv[0];
#pragma unroll
    for (int p = 1; p < nL; ++p) rLr = fma(L2[p], qv[p], rLr);
#pragma unroll
    for (int a = 1; a < D; ++a) sa = fma(Pl[a], r[a], sa);
#pragma unroll
    for (int p = 1; p < m; ++p) ss = fma(Pl[D + p], qv[p], ss);
    // y = 1/|r~| (refined estimate); |r~| = q2 y and 1/|r~|^4 = (y^2)^2
    const double y = vrsq(q2);
    const double y2 = y * y;
    const double vc = q.w * kernel_shape<KERNEL>(q2 > 0.0 ? q2 * y : 0.0);
    return vc * fma(rLr * (y2 * y2), ss, sa);
}

}  // namespace vct
