// Adjoint of the physical Laplacian operator (built on paper Eqs. lap_VCT and
// sec_SPH2; the adjoint itself is not in the paper).
//
// With lap_i = sum_{j in S_i} W_ij (phi_j - phi_i) and
//   W_ij = V_j c~_ij [P_a,i . r~_ij + (r~_ij' L~_i r~_ij) / |r~_ij|^4 P_s,i . q~_ij]
// (P_a,i, P_s,i the first- and second-order parts of particle i's Laplacian
// row of the state), the field cotangent is
//   dphi_k = sum_{i in S_k} u_i W_ik  -  sum_{j in S_k} u_k W_kj .
// Both forms below evaluate each weight once, with particle i's own state in
// registers, and sum without floating-point atomics, so every run gives the
// same bits:
//   transposed form (needs the transposed-entry map col_t): every particle i
//     writes u_i W_ij at the transposed position of its entries and its row
//     sum to a second buffer; every particle k then sums its row of the first
//     buffer in row order and subtracts its row sum;
//   push form (no map): every particle adds u_i W_ij to the accumulator of j
//     in LDS as an exact integer (below), per cell column, and the columns'
//     totals are summed per particle in a fixed order.  The bathymetry
//     adjoint with physical positions fixed (reading R2, below) sums its
//     position terms the same way.
//
// Bathymetry coefficients enter only through the VCT coefficients (projected
// positions are held fixed), so
//   dtheta_t = sum_i u_i (d c_trans_i / d coef_t) . D^ phi_i ,
// with d c_trans / d (h, h_x, h_y, h_xx, h_xy, h_yy) from forward-mode dual
// numbers, D^ phi_i from the projected-derivative rows of the forward apply,
// and d h^(k) / d coef_t the t-th term's basis products.  Per-particle
// contributions are reduced per work-group, then across work-groups, in a
// fixed order.
#include <mutex>
#include <string.h>

#include "common.h"
#include "map_dev.h"
#include "lapw.h"
#include "tiles.h"

namespace vct {

int nlist_check(const vct_nlist* nl, Grid& g);

constexpr int kALanes = 8;                     // lanes per particle
constexpr int kAThreads = kChunk * kALanes;    // one chunk per work-group
constexpr int kAWin = 1600;                    // LDS window capacity (records)

struct AdjArgs {
    int64_t n;
    double invR;
    Grid g;
    const double* pos;
    const double* vol;
    const double* state;
    const double* u;
    const double* proj;
    const int64_t* row_ptr;
    const uint16_t* col16;
    const int32_t* col_t;
    const int64_t* cs;
    const int32_t* cstart;
    const int4* cinfo;
    const int32_t* cwin;   // stored windows or NULL
    const int64_t* nchunks;
    const int64_t* chunk_off;   // [ncols + 1]: first chunk of every column
    int lap_row, nrows;
    int r_gz, r_zz, r_xz, r_yz;   // rows of dz^, z^z^, x^z^, y^z^ (-1 in 2-D) in proj
    double* partial;   // [3^(d-1)][n] per-source-column totals of the push form
    int32_t* wide;     // [2 + n / 256 + 2]: count of wide columns, longest row, list of wide columns
    double* wbuf;      // [nnz]: u_i W_ij at the transposed position
    double* rowsum;    // [n]:  u_i sum_j W_ij
    double* dphi;
    // reading R2 (physical positions fixed)
    const double* phi;   // [n] the field
    int r_pg, r_ph;      // first rows of PGRAD and PHESS in proj
    const double* gz;    // [n] d loss / d z^ through the SPH(2) derivatives (c_trans held)
    double* dzhat;       // [n] or NULL: the total d loss / d z^ (c_trans's dependence added)
    const double* r2h;   // [pairs][n] H_i of the first sweep
    const double* r2b;   // [n] bound on the row's second-sweep terms per unit volume
};

// Pass 1: u_i W_ij for every entry of row i, written transposed.  The first
// kALanes * kWSlots entries of each row (offset and transposed position) are
// loaded into registers up front; the window records are read from LDS one
// slot ahead of the arithmetic.
constexpr int kWSlots = 14;

template <int D, int KERNEL>
__global__ __launch_bounds__(kAThreads, 2) void k_adjoint_weights(AdjArgs A) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, nk = Dm::nk;
    __shared__ double4 sd[kAWin];   // x, y, z, V
    __shared__ WindowT<D> w;
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *A.nchunks) return;   // uniform over the work-group
    const int64_t n = A.n;
    const int64_t p0 = A.cstart[b], p1 = A.cstart[b + 1];
    if (threadIdx.x < kWave) {
        if (A.cwin) window_load<D>(A.cwin, b, w);
        else chunk_window_wave<D>(A.g, A.cs, A.cinfo[b], w);
    }
    const int lane = threadIdx.x % kALanes;
    const int64_t i = p0 + threadIdx.x / kALanes;
    const bool valid = i < p1;
    const int64_t ii = valid ? i : p0;
    double xi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xi[a] = a < D ? A.pos[a * n + ii] : 0.0;
    double L2[nL], Pl[nk];
    const double ui = A.u[ii];
#pragma unroll
    for (int p = 0; p < nL; ++p) L2[p] = (pair_a<D>(p) == pair_b<D>(p) ? 1.0 : 2.0) * A.state[(int64_t)p * n + ii];
#pragma unroll
    for (int c = 0; c < nk; ++c) Pl[c] = ui * A.state[(int64_t)(nL + A.lap_row * nk + c) * n + ii];
    const int64_t rb = valid ? A.row_ptr[ii] : 0, re = valid ? A.row_ptr[ii + 1] : 0;
    // register slots: entry rb + lane + kALanes s (window offset, transposed position)
    uint32_t cpk[(kWSlots + 1) / 2];
    int32_t tcol[kWSlots];
    int nslot = 0;
    {
        const uint32_t first = re > rb ? (uint32_t)A.col16[rb] : 0u;
#pragma unroll
        for (int s = 0; s < kWSlots; ++s) {
            const int64_t e = rb + lane + (int64_t)kALanes * s;
            const bool in = e < re;
            const uint32_t c = in ? (uint32_t)A.col16[e] : first;
            tcol[s] = in ? A.col_t[e] : -1;
            nslot += in ? 1 : 0;
            if (s % 2 == 0) cpk[s / 2] = c;
            else cpk[s / 2] |= c << 16;
        }
    }
    __syncthreads();
    const int W = __builtin_amdgcn_readfirstlane(w.off[w.nr]);
    auto cols = [&](int s) -> int { return dcheck((int)((cpk[s / 2] >> (16 * (s % 2))) & 0xffffu), W, kChkWindow); };
    const bool in_lds = W <= kAWin;
    if (in_lds) {
        // every load of a thread is issued before its first LDS store
        constexpr int kRep = (kAWin + kAThreads - 1) / kAThreads;
        double4 q[kRep];
#pragma unroll
        for (int k = 0; k < kRep; ++k) {
            const int t = threadIdx.x + k * kAThreads;
            if (t < W) {   // lanes past the window load nothing (whole waves skip)
                const int64_t j = window_global<D>(w, t);
                q[k] = make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
            }
        }
#pragma unroll
        for (int k = 0; k < kRep; ++k) {
            const int t = threadIdx.x + k * kAThreads;
            if (t < W) sd[t] = q[k];
        }
    }
    __syncthreads();
    auto fetch = [&](int t) -> double4 {
        t = dcheck(t, W, kChkWindow);
        if (in_lds) return sd[t];
        const int64_t j = window_global<D>(w, t);
        return make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
    };
    double sum = 0.0;
    if (in_lds) {
        double4 qn = sd[cols(0)];
#pragma unroll
        for (int s = 0; s < kWSlots; ++s) {
            const double4 q = qn;
            if (s + 1 < kWSlots) qn = sd[cols(s + 1)];
            __builtin_amdgcn_sched_barrier(0);
            if (s < nslot) {
                const double wij = lap_weight<D, KERNEL>(q, xi, A.invR, L2, Pl);
                A.wbuf[tcol[s]] = wij;
                sum += wij;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
#pragma unroll 1
        for (int s = 0; s < kWSlots; ++s) {
            if (s < nslot) {
                const double wij = lap_weight<D, KERNEL>(fetch(cols(s)), xi, A.invR, L2, Pl);
                A.wbuf[tcol[s]] = wij;
                sum += wij;
            }
        }
    }
    for (int64_t e = rb + lane + (int64_t)kALanes * kWSlots; e < re; e += kALanes) {
        const double wij = lap_weight<D, KERNEL>(fetch(A.col16[e]), xi, A.invR, L2, Pl);
        A.wbuf[A.col_t[e]] = wij;
        sum += wij;
    }
    sum = group_sum(sum, kALanes);
    if (valid && lane == 0) A.rowsum[ii] = sum;
}

// ------------------------------------------------------------------ reading R2

// With the physical positions fixed the projected heights move with the
// bathymetry, and the rows of the Laplacian change through their offsets.
// For row i write the SPH(2) system as K x = b with x = [R grad^ phi;
// R^2 D / 2], b = sum_j V_j t_ij phi_ij, K = sum_j V_j t_ij m_ij^T, t_ij =
// [c~ r~; F~ q~], m_ij = [r~; q~] and F~ = c~ (r~' L~ r~) / |r~|^4, L~ = A~^-1,
// A~ = sum_j V_j c~ r~ r~^T (the formulation of the moment kernels).  Then
// d(u_i lap_i) = u_i P_lap,i (db - dK x) (implicit differentiation), and
// b - K x = sum_j V_j t_ij psi_ij with the Taylor residual
// psi_ij = phi_ij - r~ . R grad^ phi - (1/2) r~' R^2 H^ r~.  With x held, the
// offsets enter directly and through L~; dL~ = -L~ dA~ L~ turns the latter into
// one more pair term.  So, with W_ij(r~) = V_j c~ [P_a . r~ + (r~' L~ r~)
// / |r~|^4 P_s . q~] (u_i folded into P, as in lap_weight),
//   G_i  = sum_j V_j c~ psi_ij (P_s . q~) / |r~|^4  r~ r~^T,   H_i = L~ G_i L~,
//   Phi_ij(r~) = W_ij(r~) psi_ij(r~) - V_j c~(|r~|) r~' H_i r~,
// d(u_i lap_i) / d z^_j = (1/R) d Phi_ij / d r~_z for j in S_i and minus their
// sum for j = i.  Every term is a function of one offset, so the push form
// below sums them like the Laplacian weights of the field adjoint:
// k_r2_prep runs the first sweep over each row (G_i, H_i and a bound on the
// row's terms), and the push kernels the second.

// d c~ / dq of the kernel shape (kernel_shape)
template <int KERNEL>
__device__ __forceinline__ double kernel_shape_dq(double q) {
    if (KERNEL == VCT_KERNEL_WENDLAND_C2) {
        const double t = q < 1.0 ? 1.0 - q : 0.0;
        return -3.0 * t * t;
    } else {
        const double s = 2.0 * q;
        const double t = s < 2.0 ? 2.0 - s : 0.0;
        const double outer = 2.0 * 0.75 * (-2.0 * t / s - t * t / (s * s));
        return s <= 1.0 ? -4.5 : outer;
    }
}

// One particle's row data for the position derivatives: its position and
// field value, L~ (pairs, off-diagonals doubled for the quadratic form),
// u_i P_lap, the solution at i in units of R (R grad^ phi, and the Taylor
// coefficients of (1/2) r~' R^2 H^ r~ on the pair monomials) and H_i.
template <int D> struct R2Row {
    double xi[3], phi_i;
    double L2[Dims<D>::nL], Pl[Dims<D>::nk];
    double gt[D], hh[Dims<D>::m];
    double Hm[D][D];
};

template <int D>
__device__ __forceinline__ void r2_row_load(const AdjArgs& A, int64_t ii, R2Row<D>& w) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, nk = Dm::nk, m = Dm::m;
    const int64_t n = A.n;
    const double R = 1.0 / A.invR;
#pragma unroll
    for (int a = 0; a < 3; ++a) w.xi[a] = a < D ? A.pos[a * n + ii] : 0.0;
    w.phi_i = A.phi[ii];
    const double ui = A.u[ii];
#pragma unroll
    for (int p = 0; p < nL; ++p) w.L2[p] = (pair_a<D>(p) == pair_b<D>(p) ? 1.0 : 2.0) * A.state[(int64_t)p * n + ii];
#pragma unroll
    for (int c = 0; c < nk; ++c) w.Pl[c] = ui * A.state[(int64_t)(nL + A.lap_row * nk + c) * n + ii];
    const double* pr = A.proj + ii * A.nrows;
#pragma unroll
    for (int a = 0; a < D; ++a) w.gt[a] = R * pr[A.r_pg + a];
#pragma unroll
    for (int p = 0; p < m; ++p) w.hh[p] = R * R * pr[A.r_ph + p] * (pair_a<D>(p) == pair_b<D>(p) ? 0.5 : 1.0);
}

// H_i from the first sweep's pairs
template <int D>
__device__ __forceinline__ void r2_row_h(const AdjArgs& A, int64_t ii, R2Row<D>& w) {
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int c = 0; c < D; ++c) w.Hm[a][c] = A.r2h[(int64_t)sym_index<D>(a, c) * A.n + ii];
}

// the pair quantities of both sweeps
template <int D> struct R2Pair {
    double r[D], qv[Dims<D>::m], y, y2, q, ct, sa, ss, rLr, psi, vol;
};

template <int D, int KERNEL>
__device__ __forceinline__ R2Pair<D> r2_pair(const R2Row<D>& w, const double4& qr, double ph, double invR) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, m = Dm::m;
    R2Pair<D> P;
    P.r[0] = (qr.x - w.xi[0]) * invR;
    P.r[1] = (qr.y - w.xi[1]) * invR;
    if (D == 3) P.r[D - 1] = (qr.z - w.xi[2]) * invR;
    double q2 = P.r[0] * P.r[0];
#pragma unroll
    for (int a = 1; a < D; ++a) q2 = fma(P.r[a], P.r[a], q2);
#pragma unroll
    for (int p = 0; p < m; ++p) P.qv[p] = P.r[pair_a<D>(p)] * P.r[pair_b<D>(p)];
    P.y = vrsq(q2);
    P.y2 = P.y * P.y;
    P.q = q2 > 0.0 ? q2 * P.y : 0.0;
    P.ct = kernel_shape<KERNEL>(P.q);
    P.vol = qr.w;
    double rLr = 0.0, sa = 0.0, ss = 0.0, quad = 0.0, lin = 0.0;
#pragma unroll
    for (int p = 0; p < nL; ++p) rLr = fma(w.L2[p], P.qv[p], rLr);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        sa = fma(w.Pl[a], P.r[a], sa);
        lin = fma(w.gt[a], P.r[a], lin);
    }
#pragma unroll
    for (int p = 0; p < m; ++p) {
        ss = fma(w.Pl[D + p], P.qv[p], ss);
        quad = fma(w.hh[p], P.qv[p], quad);
    }
    P.rLr = rLr; P.sa = sa; P.ss = ss;
    P.psi = (ph - w.phi_i) - lin - quad;
    return P;
}

// the second sweep's term: d Phi_ij / d z^_j
template <int D, int KERNEL>
__device__ __forceinline__ double r2_term(const R2Row<D>& w, const double4& qr, double ph, double invR) {
    using Dm = Dims<D>;
    constexpr int m = Dm::m;
    constexpr int Z = D - 1;
    const R2Pair<D> P = r2_pair<D, KERNEL>(w, qr, ph, invR);
    const double zc = P.r[Z];
    const double y4 = P.y2 * P.y2;
    const double dct = kernel_shape_dq<KERNEL>(P.q) * zc * P.y;   // d c~ / d r~_z
    double Lr = 0.0, Hr = 0.0, Htr = 0.0, rHr = 0.0;              // (L~ r~)_z, (H r~)_z, (H^~ r~)_z, r~' H r~
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int pz = sym_index<D>(Z, a);
        Lr = fma(a == Z ? w.L2[pz] : 0.5 * w.L2[pz], P.r[a], Lr);
        Hr = fma(w.Hm[Z][a], P.r[a], Hr);
        double ha = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) ha = fma(w.Hm[a][c], P.r[c], ha);
        rHr = fma(P.r[a], ha, rHr);
        // R^2 H^ from the Taylor coefficients: diagonal 2 hh, off-diagonal hh
        Htr = fma(a == Z ? 2.0 * w.hh[pz] : w.hh[pz], P.r[a], Htr);
    }
    double dss = 0.0;   // d (P_s . q~) / d r~_z
#pragma unroll
    for (int p = 0; p < m; ++p) {
        const int pa = pair_a<D>(p), pb = pair_b<D>(p);
        const double dq = (pa == Z ? P.r[pb] : 0.0) + (pb == Z ? P.r[pa] : 0.0);
        dss = fma(w.Pl[D + p], dq, dss);
    }
    const double F = P.rLr * y4;
    const double dF = 2.0 * Lr * y4 - 4.0 * P.rLr * y4 * P.y2 * zc;
    const double s1 = fma(F, P.ss, P.sa);
    const double Wv = P.vol * P.ct * s1;
    const double dW = P.vol * (dct * s1 + P.ct * (w.Pl[Z] + dF * P.ss + F * dss));
    const double dpsi = -w.gt[Z] - Htr;
    const double dZ = P.vol * (dct * rHr + 2.0 * P.ct * Hr);
    return (dW * P.psi + Wv * dpsi - dZ) * invR;
}

// First sweep per particle (one chunk per work-group, kALanes lanes per
// particle, window records and field values in LDS):
//   G_i and H_i = L~ G_i L~, written as r2h[pairs][n];
//   r2b[i], a bound on |term| / V_j over the row's terms (the push pass
//   multiplies the largest of its column by the window's largest volume):
//   with q >= q_min over the row, |r~| < 1, cmax >= c~, dcmax >= |dc~/dq|,
//   L1 = sum |L2|, Pa1 = sum |P_a|, Ps1 = sum |P_s| (|P_s . q~| <= Ps1 q^2):
//     |W| / V    <= cmax (Pa1 + L1 Ps1)
//     |dW| / V   <= dcmax (Pa1 + L1 Ps1) + cmax (Pa1 + 8 L1 Ps1 / q_min)
//     |dpsi|     <= |R dz^phi| + sum_a |R^2 H^_za|,  |psi| <= max over the row
//     |dZ| / V   <= (dcmax + 2 cmax) sum |H|
//   term <= (|dW| max|psi| + |W| |dpsi| + |dZ|) / R.
template <int D, int KERNEL>
__global__ __launch_bounds__(kAThreads, 2) void k_r2_prep(AdjArgs A, double* __restrict__ r2h,
                                                         double* __restrict__ r2b) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, m = Dm::m;
    __shared__ double4 sd[kAWin];   // x, y, z, V
    __shared__ double sf[kAWin];    // phi
    __shared__ WindowT<D> w;
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *A.nchunks) return;   // uniform over the work-group
    const int64_t n = A.n;
    const int64_t p0 = A.cstart[b], p1 = A.cstart[b + 1];
    if (threadIdx.x < kWave) {
        if (A.cwin) window_load<D>(A.cwin, b, w);
        else chunk_window_wave<D>(A.g, A.cs, A.cinfo[b], w);
    }
    __syncthreads();
    const int W = __builtin_amdgcn_readfirstlane(w.off[w.nr]);
    const bool in_lds = W <= kAWin;
    if (in_lds)
        for (int t = threadIdx.x; t < W; t += kAThreads) {
            const int64_t j = window_global<D>(w, t);
            sd[t] = make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
            sf[t] = A.phi[j];
        }
    __syncthreads();
    auto fetch = [&](int t, double& ph) -> double4 {
        t = dcheck(t, W, kChkWindow);
        if (in_lds) {
            ph = sf[t];
            return sd[t];
        }
        const int64_t j = window_global<D>(w, t);
        ph = A.phi[j];
        return make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
    };
    const int lane = threadIdx.x % kALanes;
    const int64_t i = p0 + threadIdx.x / kALanes;
    const bool valid = i < p1;
    const int64_t ii = valid ? i : p0;
    R2Row<D> row;
    r2_row_load<D>(A, ii, row);
    const int64_t rb = valid ? A.row_ptr[ii] : 0, re = valid ? A.row_ptr[ii + 1] : 0;
    double Gp[nL];
#pragma unroll
    for (int p = 0; p < nL; ++p) Gp[p] = 0.0;
    double psimax = 0.0, qmin = 2.0;
    for (int64_t e = rb + lane; e < re; e += kALanes) {
        double ph;
        const double4 qr = fetch(A.col16[e], ph);
        const R2Pair<D> P = r2_pair<D, KERNEL>(row, qr, ph, A.invR);
        const double kap = P.vol * P.ct * P.psi * P.ss * (P.y2 * P.y2);
#pragma unroll
        for (int p = 0; p < nL; ++p) Gp[p] = fma(kap, P.qv[p], Gp[p]);
        psimax = fmax(psimax, fabs(P.psi));
        qmin = fmin(qmin, P.q);
    }
#pragma unroll
    for (int p = 0; p < nL; ++p) Gp[p] = group_sum(Gp[p], kALanes);
    for (int s2 = 1; s2 < kALanes; s2 <<= 1) {
        psimax = fmax(psimax, __shfl_xor(psimax, s2, kALanes));
        qmin = fmin(qmin, __shfl_xor(qmin, s2, kALanes));
    }
    // H_i = L~ G_i L~ (symmetric; L~ off-diagonals are L2 / 2)
    double Lm[D][D], Gm[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const int p = sym_index<D>(a, c);
            Lm[a][c] = a == c ? row.L2[p] : 0.5 * row.L2[p];
            Gm[a][c] = Gp[p];
        }
    double Hp[nL];
#pragma unroll
    for (int p = 0; p < nL; ++p) {
        const int a = pair_a<D>(p), c = pair_b<D>(p);
        double t = 0.0;
#pragma unroll
        for (int e1 = 0; e1 < D; ++e1)
#pragma unroll
            for (int e2 = 0; e2 < D; ++e2) t = fma(Lm[a][e1], Gm[e1][e2] * Lm[e2][c], t);
        Hp[p] = t;
    }
    if (!valid || lane != 0) return;
#pragma unroll
    for (int p = 0; p < nL; ++p) r2h[(int64_t)p * n + i] = Hp[p];
    // the bound
    const double cmax = KERNEL == VCT_KERNEL_WENDLAND_C2 ? 1.0 : 3.0;
    const double dcmax = KERNEL == VCT_KERNEL_WENDLAND_C2 ? 3.0 : 4.5;
    double L1 = 0.0, Pa1 = 0.0, Ps1 = 0.0, Hs = 0.0, dps = fabs(row.gt[D - 1]);
#pragma unroll
    for (int p = 0; p < nL; ++p) {
        L1 += fabs(row.L2[p]);
        Hs += (pair_a<D>(p) == pair_b<D>(p) ? 1.0 : 2.0) * fabs(Hp[p]);
    }
#pragma unroll
    for (int a = 0; a < D; ++a) Pa1 += fabs(row.Pl[a]);
#pragma unroll
    for (int p = 0; p < m; ++p) Ps1 += fabs(row.Pl[D + p]);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int p = sym_index<D>(D - 1, a);
        dps += (a == D - 1 ? 2.0 : 1.0) * fabs(row.hh[p]);
    }
    const double w1 = cmax * (Pa1 + L1 * Ps1);
    const double dw1 = dcmax * (Pa1 + L1 * Ps1) + cmax * (Pa1 + 8.0 * L1 * Ps1 / qmin);
    const double dz1 = (dcmax + 2.0 * cmax) * Hs;
    r2b[i] = (dw1 * psimax + w1 * dps + dz1) * A.invR;
}

// Push form (no transposed map).  Every particle i evaluates u_i W_ij once
// for each entry of its own row, with its state in registers, and adds it to
// the accumulator of j; particle j receives these from the particles of the
// 3^(d-1) cell columns around its own.  One work-group takes one cell column:
// its accumulators cover the column's window (every particle of the
// neighbouring columns, all z cells) in LDS, next to the window's records.
// The self term -u_i sum_j W_ij is added at particle i's own accumulator.  At
// the end the column writes, for every particle j of its window, its total
// into slot s of j (s = position of j's column relative to the source
// column), and k_adjoint_combine sums the slots of each particle in a fixed
// order.
//
// The accumulation is exact and order-free.  With a per-column bound M on the
// terms (below) and d_max the longest row of the set, every term w is scaled
// by 2^k, k = 61 - ilogb(M) - bitlen(2 d_max), rounded to the integer
// X = rint(w 2^k), and added by a 64-bit integer atomic.  The accumulator of
// particle j receives at most one term per neighbour of j (the neighbour
// relation is symmetric) and one self term of at most d_max M, so its sum
// stays below 2^63; integer sums do not depend on the order of arrival, so
// the result has the same bits on every run.  The total is converted once to
// FP64 and scaled back.  The resolution 2^-k is at most 2^-52 d_max M, about
// one FP64 rounding of a sum of d_max terms of size M.  (A coarser 2^-50 M,
// which a one-instruction rounding would allow, loses terms far below the
// bound systematically: the R2 sums then drift by parts in 1e10.)
//
// Bound: with r~ = r/R (|r~| < 1 inside the support), |q~_p| <= |r~|^2 and
// |r~' L~ r~| <= (sum |L~|) |r~|^2, so for the kernel shape c~ <= c_max
//   |u_i W_ij| <= V_j c_max (sum_a |u P_a,i| + (sum |L~_i|) (sum_p |u P_s,i|)).
constexpr int kPThreads = 1024;   // 128 particles at a time, 8 lanes each (the field adjoint)
constexpr int kPAcc = 3840;       // accumulators (and staged records) per pass over a column's window
constexpr int kPChunks = 24;      // chunk windows of one column held in LDS
constexpr int kPSlots = 16;       // row entries per lane loaded into registers at a time
// the int32 side buffer of the push form: count of wide columns, longest row, list of wide columns
constexpr int kWideCount = 0, kWideMaxDeg = 1, kWideList = 2;

// X = rint(x) as a 64-bit integer when |X| < 2^62 (then true); false for a
// value out of range or not finite
__device__ __forceinline__ bool quantize(double x, unsigned long long& X) {
    const double xs = rint(x);
    const bool ok = fabs(xs) < 0x1p62;
    const double v = ok ? xs : 0.0;
    const double hd = floor(v * 0x1p-32);                       // |hd| < 2^30
    const unsigned int l = (unsigned int)fma(hd, -0x1p32, v);   // exact, in [0, 2^32)
    X = ((unsigned long long)(unsigned int)(int)hd << 32) | l;
    return ok;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
    for (int m = 1; m < kWave; m <<= 1) {
        const T o = __shfl_xor(v, m, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// What the push form sums: the Laplacian weights u_i W_ij of the field
// adjoint, or the position terms d Phi_ij / d z^_j of reading R2 (these read
// the field values too, staged with the records).
// R2 runs half the threads: its rows hold about twice the registers.  With
// two waves per SIMD it also reads the range shifts of a piece of entries up
// front (kShiftWin), which the Laplacian's four waves do not gain from.
struct PushLap {
    static constexpr int kAcc = kPAcc, kThreads = kPThreads;
    static constexpr bool kR2 = false, kShiftWin = false;
};
struct PushR2 {
    static constexpr int kAcc = 3200, kThreads = kPThreads / 2;
    static constexpr bool kR2 = true, kShiftWin = true;
};

// One column.  FAST = true handles a column whose window fits the
// accumulators (one pass, records in LDS) and appends any other column to the
// list `wide` ([0] = count); FAST = false handles a listed column (passes over
// the window, records read from memory).
template <int D, int KERNEL, class OP, bool FAST>
__device__ __forceinline__ void push_column(const AdjArgs& A, double* __restrict__ partial, int64_t c,
                                            int32_t* __restrict__ wide) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, nk = Dm::nk, m = Dm::m;
    constexpr int NS = D == 3 ? 9 : 3;
    constexpr int kThreads = OP::kThreads;
    constexpr int kW = kThreads / kWave;
    constexpr int kAcc = OP::kAcc;
    __shared__ unsigned long long s_acc[kAcc];
    __shared__ double4 s_pos[FAST ? kAcc : 1];
    __shared__ double s_phi[FAST && OP::kR2 ? kAcc : 1];
    __shared__ uint32_t s_nan[kAcc / 32];
    __shared__ WindowT<D> s_cw;
    __shared__ WindowT<D> s_chw[kPChunks];
    // per chunk of the current group: range starts in its window (INT_MAX past
    // the last range) and the shift from its window to the column window
    __shared__ int s_off[kPChunks][kMaxRanges + 1];
    __shared__ int s_sh[kPChunks][kMaxRanges];
    __shared__ int s_slot[kMaxRanges];
    __shared__ double s_red[2][kW];

    const int64_t n = A.n;
    const int tid = threadIdx.x;
    const int wv = tid / kWave;
    const int64_t nz = grid_nz<D>(A.g);
    const int64_t b0 = A.chunk_off[c], b1 = A.chunk_off[c + 1];
    const int nch = (int)(b1 - b0);
    if (wv == 0) {
        chunk_window_wave<D>(A.g, A.cs, make_int4((int)c, 0, (int)(nz - 1), 0), s_cw);
    } else if (tid == kWave) {
        // relative position of every range's column, in the order of the ranges
        int r = 0;
        for (int sl = 0; sl < NS; ++sl) {
            int64_t x, y = 0;
            if (D == 3) { x = c / A.g.nc[1] + sl / 3 - 1; y = c % A.g.nc[1] + sl % 3 - 1; }
            else x = c + sl - 1;
            if (x >= 0 && x < A.g.nc[0] && (D == 2 || (y >= 0 && y < A.g.nc[1]))) s_slot[r++] = sl;
        }
    }
    __syncthreads();
    const int Wc = s_cw.off[s_cw.nr];
    if (FAST && Wc > kAcc) {   // uniform: left to the wide pass
        if (tid == 0) wide[kWideList + atomicAdd(&wide[kWideCount], 1)] = (int32_t)c;
        return;
    }
    int rown = 0;   // the column's own range
    for (int r = 0; r < kMaxRanges; ++r)
        if (r < s_cw.nr && s_slot[r] == NS / 2) rown = r;
    const int64_t q0 = s_cw.gstart[rown];

    // records of the whole window in LDS (FAST), and the column's scale: the
    // largest volume of the window, the largest per-particle bound and the
    // longest row of the column's particles
    double vmax = 0.0, bmax = 0.0;
    for (int t = tid; t < Wc; t += kThreads) {
        const int64_t j = window_global<D>(s_cw, t);
        const double v = A.vol[j];
        vmax = fmax(vmax, v);
        if (FAST) s_pos[t] = make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, v);
        if (FAST && OP::kR2) s_phi[t] = A.phi[j];
    }
    // the first group of chunk windows, loaded alongside
    for (int cb = wv; cb < (nch < kPChunks ? nch : kPChunks); cb += kW)
        window_load<D>(A.cwin, (uint32_t)(b0 + cb), s_chw[cb]);
    const int qlen = s_cw.off[rown + 1] - s_cw.off[rown];
    for (int q = tid; q < qlen; q += kThreads) {
        const int64_t i = q0 + q;
        double bnd;
        if constexpr (OP::kR2) {
            bnd = A.r2b[i];
        } else {
            double sL = 0.0, sa = 0.0, ss = 0.0;
#pragma unroll
            for (int p = 0; p < nL; ++p) sL += (pair_a<D>(p) == pair_b<D>(p) ? 1.0 : 2.0) * fabs(A.state[(int64_t)p * n + i]);
#pragma unroll
            for (int a = 0; a < D; ++a) sa += fabs(A.state[(int64_t)(nL + A.lap_row * nk + a) * n + i]);
#pragma unroll
            for (int p = 0; p < m; ++p) ss += fabs(A.state[(int64_t)(nL + A.lap_row * nk + D + p) * n + i]);
            bnd = fabs(A.u[i]) * (sa + sL * ss);
        }
        if (bnd <= 1.7976931348623157e308) bmax = fmax(bmax, bnd);   // skips NaN and infinity
    }
    vmax = wave_max(vmax);
    bmax = wave_max(bmax);
    if (tid % kWave == 0) {
        s_red[0][wv] = vmax;
        s_red[1][wv] = bmax;
    }
    __syncthreads();
    vmax = 0.0;
    bmax = 0.0;
#pragma unroll
    for (int w = 0; w < kW; ++w) {
        vmax = fmax(vmax, s_red[0][w]);
        bmax = fmax(bmax, s_red[1][w]);
    }
    // (the R2 bound already holds the kernel-shape factors)
    const double cmax = OP::kR2 ? 1.0 : KERNEL == VCT_KERNEL_WENDLAND_C2 ? 1.0 : 3.0;
    const double Mb = vmax * cmax * 1.0625 * bmax;   // the factor covers |r~| rounded above 1
    // terms reaching one accumulator: at most one per neighbour of its
    // particle, plus the self term of at most (longest row) x M
    const double nterm = 2.0 * (double)wide[kWideMaxDeg];
    const int k = (Mb > 0.0 && Mb <= 1.7976931348623157e308) ? 61 - ilogb(Mb) - (ilogb(fmax(nterm, 1.0)) + 1) : 0;

    const int lane = tid % kALanes;
    const int slot = tid / kALanes;
    constexpr int kBatch = kThreads / kALanes;

    // one particle's row
    auto rows = [&](int cb, int64_t ii, bool valid, int q, int t0, int tn) {
        R2Row<D> row;
        if constexpr (OP::kR2) {
            r2_row_load<D>(A, ii, row);
            r2_row_h<D>(A, ii, row);
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) row.xi[a] = a < D ? A.pos[a * n + ii] : 0.0;
            const double ui = A.u[ii];
#pragma unroll
            for (int p = 0; p < nL; ++p)
                row.L2[p] = (pair_a<D>(p) == pair_b<D>(p) ? 1.0 : 2.0) * A.state[(int64_t)p * n + ii];
#pragma unroll
            for (int cc = 0; cc < nk; ++cc) row.Pl[cc] = ui * A.state[(int64_t)(nL + A.lap_row * nk + cc) * n + ii];
        }
        const int tci = s_cw.off[rown] + q - t0;   // the particle's own accumulator
        const bool self_in = valid && (FAST || (unsigned)tci < (unsigned)tn);
        const int64_t rb = valid ? A.row_ptr[ii] : 0, re = valid ? A.row_ptr[ii + 1] : 0;
        // every lane takes a contiguous block of the row
        const int nb = (int)((re - rb + kALanes - 1) / kALanes);
        const int64_t lb = rb + (int64_t)lane * nb;
        const int64_t le = lb + nb < re ? lb + nb : re;
        // range cursor: the entries ascend, so the range only moves forward;
        // it starts at the range of the block's first entry
        int r = 0;
        if (lb < le) {
            const int t0e = A.col16[lb];
#pragma unroll
            for (int kk = 1; kk < kMaxRanges; ++kk) r += t0e >= s_off[cb][kk] ? 1 : 0;
        }
        int nxt = s_off[cb][r + 1];
        int sh = s_sh[cb][r];
        auto column_offset = [&](int t) {   // window offset of the chunk -> of the column
            while (t >= nxt) {
                ++r;
                nxt = s_off[cb][r + 1];
                sh = s_sh[cb][r];
            }
            return t + sh;
        };
        double rowsum = 0.0;
        // the block in pieces of kPSlots entries, each piece's offsets loaded
        // together (two 16-bit offsets per register) before any is used
        for (int64_t eb = lb; eb < le; eb += kPSlots) {
            const int cnt = (int)(le - eb < kPSlots ? le - eb : kPSlots);
            uint32_t cpk[kPSlots / 2];
            const uint16_t* cp = A.col16 + eb;
#pragma unroll
            for (int s2 = 0; s2 < kPSlots; ++s2) {
                // with kShiftWin the slots past the block's end re-read its
                // last entry (no branch; the last slot then holds that entry)
                uint32_t cv;
                if (OP::kShiftWin) cv = cp[(uint32_t)(s2 < cnt ? s2 : cnt - 1)];
                else cv = s2 < cnt ? (uint32_t)cp[s2] : 0u;
                if (s2 % 2 == 0) cpk[s2 / 2] = cv;
                else cpk[s2 / 2] |= cv << 16;
            }
            // FAST: the shifts of the ranges of the piece's first entry and the
            // three after it, read together; a piece that reaches further (a
            // few in a thousand) moves the cursor entry by entry instead
            int b1 = 0, b2 = 0, b3 = 0, h0 = 0, h1 = 0, h2 = 0, h3 = 0;
            bool fastp = false;
            if (FAST && OP::kShiftWin) {
                const int tf = (int)(cpk[0] & 0xffffu), tl = (int)(cpk[kPSlots / 2 - 1] >> 16);   // first, last
                while (tf >= nxt) {
                    ++r;
                    nxt = s_off[cb][r + 1];
                    sh = s_sh[cb][r];
                }
                auto off_at = [&](int m) { return s_off[cb][r + m < kMaxRanges ? r + m : kMaxRanges]; };
                auto sh_at = [&](int m) { return s_sh[cb][r + m < kMaxRanges - 1 ? r + m : kMaxRanges - 1]; };
                b1 = nxt; b2 = off_at(2); b3 = off_at(3);
                h0 = sh; h1 = sh_at(1); h2 = sh_at(2); h3 = sh_at(3);
                fastp = tl < off_at(4);
            }
            // fully unrolled: the slots past the block's end are masked
#pragma unroll
            for (int s2 = 0; s2 < kPSlots; ++s2) {
                if (s2 < cnt) {
                    const int t = (int)((cpk[s2 / 2] >> (16 * (s2 % 2))) & 0xffffu);
                    int tg;
                    if (FAST && OP::kShiftWin) {
                        int hs = h0;
                        hs = t >= b1 ? h1 : hs;
                        hs = t >= b2 ? h2 : hs;
                        hs = t >= b3 ? h3 : hs;
                        tg = fastp ? t + hs : column_offset(t);
                    } else {
                        tg = column_offset(t);
                    }
                    tg = dcheck(tg, Wc, kChkAccum);
                    const int tc = tg - t0;
                    const bool here = FAST || (unsigned)tc < (unsigned)tn;
                    if (here || self_in) {
                        double4 qv;
                        double ph = 0.0;
                        if (FAST) {
                            qv = s_pos[tg];
                            if (OP::kR2) ph = s_phi[tg];
                        } else {
                            const int64_t j = s_cw.gstart[r] + (tg - s_cw.off[r]);
                            qv = make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
                            if (OP::kR2) ph = A.phi[j];
                        }
                        double wij;
                        if constexpr (OP::kR2) wij = r2_term<D, KERNEL>(row, qv, ph, A.invR);
                        else wij = lap_weight<D, KERNEL>(qv, row.xi, A.invR, row.L2, row.Pl);
                        rowsum += wij;
                        if (here) {
                            unsigned long long X;
                            if (quantize(ldexp(wij, k), X)) atomicAdd(&s_acc[tc], X);
                            else atomicOr(&s_nan[tc >> 5], 1u << (tc & 31));
                        }
                    }
                }
            }
        }
        rowsum = group_sum(rowsum, kALanes);
        if (self_in && lane == 0) {
            unsigned long long X;
            if (quantize(ldexp(-rowsum, k), X)) atomicAdd(&s_acc[tci], X);
            else atomicOr(&s_nan[tci >> 5], 1u << (tci & 31));
        }
    };

    // passes over the column window (one unless it exceeds the accumulators)
    for (int t0 = 0; t0 < Wc; t0 += kAcc) {
        const int tn = Wc - t0 < kAcc ? Wc - t0 : kAcc;
        for (int t = tid; t < tn; t += kThreads) s_acc[t] = 0ull;
        for (int t = tid; t < (tn + 31) / 32; t += kThreads) s_nan[t] = 0u;
        // the column's chunks, kPChunks at a time
        for (int g0 = 0; g0 < nch; g0 += kPChunks) {
            const int ncl = nch - g0 < kPChunks ? nch - g0 : kPChunks;
            if (g0 > 0 || (t0 > 0 && nch > kPChunks)) {   // else the prologue loaded them
                __syncthreads();   // the previous group's tables consumed
                for (int cb = wv; cb < ncl; cb += kW) window_load<D>(A.cwin, (uint32_t)(b0 + g0 + cb), s_chw[cb]);
            }
            __syncthreads();   // windows loaded; accumulators cleared
            if (tid < ncl * (kMaxRanges + 1)) {
                const int cb = tid / (kMaxRanges + 1), r = tid % (kMaxRanges + 1);
                const WindowT<D>& w = s_chw[cb];   // both windows list the same columns in the same order
                s_off[cb][r] = r < w.nr ? w.off[r] : INT_MAX;
                if (r < kMaxRanges)
                    s_sh[cb][r] = r < w.nr ? s_cw.off[r] - w.off[r] + (int)(w.gstart[r] - s_cw.gstart[r]) : 0;
            }
            __syncthreads();
            const int qa = (int)(A.cstart[b0 + g0] - q0), qb = (int)(A.cstart[b0 + g0 + ncl] - q0);
            // the group's particles, 128 at a time; the waves run independently
            for (int q = qa + slot; q - slot < qb; q += kBatch) {
                const bool valid = q < qb;
                const int64_t ii = q0 + (valid ? q : qa);
                int cb = 0;   // the particle's chunk within the group
                for (int kk = 1; kk < ncl; ++kk)
                    if ((int64_t)A.cstart[b0 + g0 + kk] <= ii) cb = kk;
                rows(cb, ii, valid, q, t0, tn);
            }
        }
        __syncthreads();
        // this pass's totals, into the slot of each destination
        for (int t = tid; t < tn; t += kThreads) {
            const int tt = t0 + t;
            int r = 0;
#pragma unroll
            for (int kk = 1; kk < kMaxRanges; ++kk)
                if (kk < s_cw.nr && tt >= s_cw.off[kk]) r = kk;
            const int64_t j = s_cw.gstart[r] + (tt - s_cw.off[r]);
            const unsigned long long X = s_acc[t];
            const double hv = (double)(int)(unsigned int)(X >> 32), lv = (double)(unsigned int)X;
            double v = ldexp(fma(hv, 0x1p32, lv), -k);
            if ((s_nan[t >> 5] >> (t & 31)) & 1u) v = __builtin_nan("");
            partial[(int64_t)s_slot[r] * n + j] = v;
        }
        __syncthreads();
    }
}

template <int D, int KERNEL, class OP>
__global__ __launch_bounds__(OP::kThreads, 1) void k_adjoint_push(AdjArgs A, double* __restrict__ partial,
                                                               int32_t* __restrict__ wide) {
    const int64_t c = xcd_tile(blockIdx.x, gridDim.x);
    if (c >= grid_ncols<D>(A.g)) return;   // uniform over the work-group
    push_column<D, KERNEL, OP, true>(A, partial, c, wide);
}

// the listed wide columns, taken in turn by a fixed grid
template <int D, int KERNEL, class OP>
__global__ __launch_bounds__(OP::kThreads, 1) void k_adjoint_push_wide(AdjArgs A, double* __restrict__ partial,
                                                                    int32_t* __restrict__ wide) {
    const int cnt = wide[kWideCount];
    for (int w = blockIdx.x; w < cnt; w += gridDim.x) {
        push_column<D, KERNEL, OP, false>(A, partial, wide[kWideList + w], wide);
        __syncthreads();
    }
}

// the longest row of the set, into wide[kWideMaxDeg] (zeroed before)
__global__ __launch_bounds__(256) void k_adjoint_maxdeg(int64_t n, const int64_t* __restrict__ row_ptr,
                                                        int32_t* __restrict__ wide) {
    int d = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t di = row_ptr[i + 1] - row_ptr[i];
        d = di > d ? (int)(di < INT_MAX ? di : INT_MAX) : d;
    }
    d = wave_max(d);
    if (threadIdx.x % kWave == 0) atomicMax(&wide[kWideMaxDeg], d);
}

__global__ void k_zero_wide(int32_t* p) {
    p[kWideCount] = 0;
    p[kWideMaxDeg] = 0;
}

// dphi_j = sum of the slots of j, in slot order, over the source columns that
// exist (the column of j minus each relative position)
template <int D>
__global__ __launch_bounds__(256) void k_adjoint_combine(int64_t n, Grid g, const double* __restrict__ pos,
                                                         const double* __restrict__ partial,
                                                         double* __restrict__ dphi) {
    constexpr int NS = D == 3 ? 9 : 3;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t cx = cell_coord(pos[j], g.lo[0], g.inv_cs[0], g.nc[0]);
    const int64_t cy = D == 3 ? cell_coord(pos[n + j], g.lo[1], g.inv_cs[1], g.nc[1]) : 0;
    double s = 0.0;
#pragma unroll
    for (int sl = 0; sl < NS; ++sl) {
        const int64_t sx = cx - (D == 3 ? sl / 3 - 1 : sl - 1);
        const int64_t sy = cy - (D == 3 ? sl % 3 - 1 : 0);
        if (sx >= 0 && sx < g.nc[0] && (D == 2 || (sy >= 0 && sy < g.nc[1]))) s += partial[(int64_t)sl * n + j];
    }
    dphi[j] = s;
}

// Pass 2: dphi_k = (row k of the transposed buffer, summed in row order) - rowsum_k.
__global__ __launch_bounds__(256) void k_adjoint_gather(int64_t n, const int64_t* __restrict__ row_ptr,
                                                        const double* __restrict__ wbuf,
                                                        const double* __restrict__ rowsum,
                                                        double* __restrict__ dphi) {
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kALanes;
    const int lane = threadIdx.x % kALanes;
    const bool valid = k < n;
    double s = 0.0;
    if (valid) {
        const int64_t rb = row_ptr[k], re = row_ptr[k + 1];
        for (int64_t e = rb + lane; e < re; e += kALanes) s += wbuf[e];
    }
    s = group_sum(s, kALanes);
    if (valid && lane == 0) dphi[k] = s - rowsum[k];
}

constexpr int kRedThreads = 256;

// dtheta, first level.  Per particle (one thread): the projected derivatives
// that c_trans weights, from the rows of the forward apply, then
// xi_q = u_i d(c_trans . D^)/d h^(q) for the six bottom quantities h^ (dual
// numbers through the mapping coefficients), and for every bathymetry term t
// the contribution sum_q xi_q dh^(q)/dcoef_t.  With the separable table the
// terms' factor products come from the factors evaluated once per particle,
// one sum per factor pair (X_a, Y_b) that some term uses; otherwise term by
// term.  Each sum is taken over a wave (fixed lane order), the waves' sums in
// wave order: one partial per work-group and term.
template <int D, bool R2 = false>
__global__ __launch_bounds__(kRedThreads) void k_dtheta_partials(AdjArgs A, MapParams mp,
                                                                  double* __restrict__ partials) {
    constexpr int kW = kRedThreads / kWave;
    constexpr int kSlots = kMapFn * kMapFn > VCT_MAX_TERMS ? kMapFn * kMapFn : VCT_MAX_TERMS;
    __shared__ double red[kW][kSlots];
    const int64_t n = A.n;
    const int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x;
    const bool valid = i < n;
    double x[D];
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = valid ? A.pos[a * n + i] : 0.0;
    const double xs = x[0], ys = D == 3 ? x[1] : 0.0;
    SepFactors F;
    double h[6];
    if (mp.sep) {
        sep_table(mp, xs, ys, F);
        bottom6_sep(mp, F, h);
    } else {
        bottom6(mp, xs, ys, h);
    }
    double xv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (valid) {
        const double* pr = A.proj + i * A.nrows;
        const double gz = pr[A.r_gz];
        const double Hzz = pr[A.r_zz];
        const double Hxz = pr[A.r_xz];
        const double Hyz = (D == 3) ? pr[A.r_yz] : 0.0;
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
            xv[q] = ui * (mc.c0.d[q] * gz + mc.c3.d[q] * Hzz + mc.c4.d[q] * Hxz + mc.c5.d[q] * Hyz);
        if (R2) {
            // reading R2: z^ = alpha (z + beta) moves with the bottom at fixed z.
            // The total d loss / d z^ adds c_trans's own dependence on z^ (through
            // z + beta = z^ / alpha) to the SPH(2) part, and every bottom quantity
            // reaches it through d z^ / d h^(q) = alpha_q (z + beta) + alpha beta_q.
            const double a = mc.alpha.v, zb = x[D - 1] / a, ia = 1.0 / a;
            const double ax = mc.zxz.v, ay = mc.zyz.v;
            const double dc0 = (mc.axx.v + mc.ayy.v) * ia;
            const double dc3 = 2.0 * (mc.gx.v * ax + mc.gy.v * ay) * ia;
            const double dc4 = 2.0 * ax * ia, dc5 = 2.0 * ay * ia;
            const double gzt = A.gz[i] + ui * (dc0 * gz + dc3 * Hzz + dc4 * Hxz + dc5 * Hyz);
            if (A.dzhat) A.dzhat[i] = gzt;
#pragma unroll
            for (int q = 0; q < 6; ++q) xv[q] += gzt * (mc.alpha.d[q] * zb + a * mc.beta.d[q]);
        }
    }
    const int wv = threadIdx.x / kWave;
    const bool lead = threadIdx.x % kWave == 0;
    // uniform loops: every lane takes part in the wave sums
    if (mp.sep) {
#pragma unroll
        for (int a = 0; a < kMapFn; ++a) {
            if (a >= mp.nfx) break;
#pragma unroll
            for (int b = 0; b < kMapFn; ++b) {
                if (b >= mp.nfy) break;
                double v = xv[0] * (F.X0[a] * F.Y0[b]);
                v += xv[1] * (F.X1[a] * F.Y0[b]);
                v += xv[2] * (F.X0[a] * F.Y1[b]);
                v += xv[3] * (F.X2[a] * F.Y0[b]);
                v += xv[4] * (F.X1[a] * F.Y1[b]);
                v += xv[5] * (F.X0[a] * F.Y2[b]);
                v = group_sum(v, kWave);
                if (lead) red[wv][a * kMapFn + b] = v;
            }
        }
    } else {
        for (int t = 0; t < mp.nterms; ++t) {
            double v = 0.0;
            if (valid) {
                double o[6];
                term_derivs(mp, t, xs, ys, o);
#pragma unroll
                for (int q = 0; q < 6; ++q) v += xv[q] * o[q];
            }
            v = group_sum(v, kWave);
            if (lead) red[wv][t] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < mp.nterms) {
        const int t = threadIdx.x;
        const int slot = mp.sep ? mp.term_a[t] * kMapFn + mp.term_b[t] : t;
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kW; ++w) v += red[w][slot];
        partials[(int64_t)blockIdx.x * mp.nterms + t] = v;
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

// A second stream of the calling thread on the current device (default
// priority), with the two events of a fork and join, made on first use and
// kept until the process ends: the d/dtheta reduction, which only reads the
// inputs, runs there beside the d/dphi kernels.  Per thread, so calls from
// several host threads do not share the events.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
static int side_stream(SideStream** out) {
    constexpr int kDev = 64;
    thread_local SideStream side[kDev];
    int dev = -1;
    VCT_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kDev) return VCT_E_ARG;
    SideStream& ss = side[dev];
    if (!ss.s) {
        VCT_HIP_CHECK(hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming));
        VCT_HIP_CHECK(hipEventCreateWithFlags(&ss.join, hipEventDisableTiming));
        VCT_HIP_CHECK(hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking));
    }
    *out = &ss;
    return VCT_OK;
}

template <int D>
static int launch_dtheta(const AdjArgs& a, const MapParams& mp, double* dtheta, double* partials, hipStream_t s) {
    const int64_t nred = (a.n + kRedThreads - 1) / kRedThreads;
    VCT_LAUNCH("k_dtheta_partials", (k_dtheta_partials<D>), dim3((unsigned)nred), dim3(kRedThreads), 0, s, a, mp,
               partials);
    VCT_LAUNCH_CHECK();
    VCT_LAUNCH("k_dtheta_final", k_dtheta_final, dim3((unsigned)mp.nterms), dim3(kRedThreads), 0, s, nred,
               mp.nterms, partials, dtheta);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

// overlap: run d/dtheta on the calling thread's second stream, forked from
// and joined back into s (not for the allocation-free entry point, whose
// first call must not create streams)
template <int D, int KERNEL>
static int launch_adjoint(AdjArgs a, int64_t cap, const MapParams& mp, double* dtheta, double* partials,
                          bool overlap, hipStream_t s) {
    const int64_t n = a.n;
    const bool want_dtheta = dtheta && mp.nterms > 0;
    SideStream* side = nullptr;
    if (overlap && want_dtheta && a.dphi) {
        int st = side_stream(&side);
        if (st) return st;
        VCT_HIP_CHECK(hipEventRecord(side->fork, s));
        VCT_HIP_CHECK(hipStreamWaitEvent(side->s, side->fork, 0));
        st = launch_dtheta<D>(a, mp, dtheta, partials, side->s);
        if (st) return st;
        VCT_HIP_CHECK(hipEventRecord(side->join, side->s));
    }
    if (a.dphi && a.col_t) {
        VCT_LAUNCH("k_adjoint_weights", (k_adjoint_weights<D, KERNEL>), dim3((unsigned)cap), dim3(kAThreads), 0, s, a);
        VCT_LAUNCH_CHECK();
        VCT_LAUNCH("k_adjoint_gather", k_adjoint_gather, dim3((unsigned)((n * kALanes + 255) / 256)), dim3(256), 0,
                   s, n, a.row_ptr, a.wbuf, a.rowsum, a.dphi);
        VCT_LAUNCH_CHECK();
    } else if (a.dphi) {
        const int64_t ncols = D == 3 ? a.g.nc[0] * a.g.nc[1] : a.g.nc[0];
        VCT_LAUNCH("k_zero_wide", k_zero_wide, dim3(1), dim3(1), 0, s, a.wide);
        VCT_LAUNCH_CHECK();
        VCT_LAUNCH("k_adjoint_maxdeg", k_adjoint_maxdeg, dim3(512), dim3(256), 0, s, n, a.row_ptr, a.wide);
        VCT_LAUNCH_CHECK();
        VCT_LAUNCH("k_adjoint_push", (k_adjoint_push<D, KERNEL, PushLap>), dim3((unsigned)ncols), dim3(PushLap::kThreads),
                   0, s, a, a.partial, a.wide);
        VCT_LAUNCH_CHECK();
        VCT_LAUNCH("k_adjoint_push (wide)", (k_adjoint_push_wide<D, KERNEL, PushLap>), dim3(256), dim3(PushLap::kThreads), 0,
                   s, a, a.partial, a.wide);
        VCT_LAUNCH_CHECK();
        VCT_LAUNCH("k_adjoint_combine", (k_adjoint_combine<D>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                   n, a.g, a.pos, a.partial, a.dphi);
        VCT_LAUNCH_CHECK();
    }
    if (side) {
        VCT_HIP_CHECK(hipStreamWaitEvent(s, side->join, 0));
    } else if (want_dtheta) {
        const int st = launch_dtheta<D>(a, mp, dtheta, partials, s);
        if (st) return st;
    }
    return VCT_OK;
}

template <int D, int KERNEL>
static int launch_r2(AdjArgs a, int64_t cap, const MapParams& mp, double* gz, double* dtheta, double* partials,
                     double* r2h, double* r2b, hipStream_t s) {
    const int64_t n = a.n;
    const int64_t ncols = D == 3 ? a.g.nc[0] * a.g.nc[1] : a.g.nc[0];
    VCT_LAUNCH("k_zero_wide", k_zero_wide, dim3(1), dim3(1), 0, s, a.wide);
    VCT_LAUNCH_CHECK();
    VCT_LAUNCH("k_adjoint_maxdeg", k_adjoint_maxdeg, dim3(512), dim3(256), 0, s, n, a.row_ptr, a.wide);
    VCT_LAUNCH_CHECK();
    VCT_LAUNCH("k_r2_prep", (k_r2_prep<D, KERNEL>), dim3((unsigned)cap), dim3(kAThreads), 0, s, a, r2h, r2b);
    VCT_LAUNCH_CHECK();
    a.r2h = r2h;
    a.r2b = r2b;
    VCT_LAUNCH("k_adjoint_push (R2)", (k_adjoint_push<D, KERNEL, PushR2>), dim3((unsigned)ncols), dim3(PushR2::kThreads), 0,
               s, a, a.partial, a.wide);
    VCT_LAUNCH_CHECK();
    VCT_LAUNCH("k_adjoint_push (R2, wide)", (k_adjoint_push_wide<D, KERNEL, PushR2>), dim3(256), dim3(PushR2::kThreads), 0,
               s, a, a.partial, a.wide);
    VCT_LAUNCH_CHECK();
    VCT_LAUNCH("k_adjoint_combine", (k_adjoint_combine<D>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
               a.g, a.pos, a.partial, gz);
    VCT_LAUNCH_CHECK();
    a.gz = gz;
    const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
    VCT_LAUNCH("k_dtheta_partials (R2)", (k_dtheta_partials<D, true>), dim3((unsigned)nred), dim3(kRedThreads), 0, s,
               a, mp, partials);
    VCT_LAUNCH_CHECK();
    if (dtheta && mp.nterms > 0) {
        VCT_LAUNCH("k_dtheta_final", k_dtheta_final, dim3((unsigned)mp.nterms), dim3(kRedThreads), 0, s, nred,
                   mp.nterms, partials, dtheta);
        VCT_LAUNCH_CHECK();
    }
    return VCT_OK;
}

__global__ void k_zero_f64(double* p, int64_t cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = 0.0;
}

VCT_CHECKS_TU(checks_adjoint)

}  // namespace vct

using namespace vct;

// Columns whose window exceeds the accumulators (at least 3200 particles):
// each particle lies in at most 3^(d-1) <= 9 windows, so there are fewer than
// 9 n / 3200 < n / 256 of them.
static int64_t wide_list_len(int64_t n) { return n / 256 + 2; }

extern "C" size_t vct_adjoint_workspace_size(int dim, int64_t n, int64_t nnz, int nterms) {
    if ((dim != 2 && dim != 3) || n < 0 || nnz < 0 || nterms < 0) return 0;
    const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
    const int ns = dim == 3 ? 9 : 3;
    return aligned_sum({(size_t)(nred > 0 ? nred : 1) * (nterms > 0 ? nterms : 1) * 8,
                        (size_t)(nnz > 0 ? nnz : 1) * sizeof(double), (size_t)(n > 0 ? n : 1) * sizeof(double),
                        (size_t)(n > 0 ? n : 1) * ns * sizeof(double), (size_t)(wide_list_len(n) + kWideList) * 4});
}

// The body of both adjoint entry points; push_only ignores a transposed-entry
// map (the allocation-free variant has no room for its entry buffer).
static int adjoint_run(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                       const double* state64, uint32_t out_mask, const vct_map* map, const double* proj,
                       const double* u, double* dphi, double* dtheta, void* ws, size_t ws_bytes, bool push_only,
                       void* stream) {
    // the Laplacian row, and dz^, z^z^, x^z^ (y^z^) from PZ or from PGRAD + PHESS
    const bool pz = (out_mask & VCT_OUT_PZ) != 0;
    const bool pgh = (out_mask & (VCT_OUT_PGRAD | VCT_OUT_PHESS)) == (VCT_OUT_PGRAD | VCT_OUT_PHESS);
    Grid g;
    int st = nlist_check(nl, g);
    if (st) return st;
    const int dim = nl->dim;
    const int64_t n = nl->n;
    if (!map || !mask_valid(out_mask) || !(out_mask & VCT_OUT_LAP) || !(pz || pgh) ||
        (kernel != VCT_KERNEL_WENDLAND_C2 && kernel != VCT_KERNEL_CUBIC_SPLINE))
        return VCT_E_ARG;
    MapParams mp;
    st = map_params_from(map, dim, n, mp);
    if (st) return st;
    hipStream_t s = as_stream(stream);
    if (n == 0) {
        if (dtheta && mp.nterms > 0) {
            VCT_LAUNCH("k_zero_f64", k_zero_f64, dim3(1), dim3(64), 0, s, dtheta, (int64_t)mp.nterms);
            VCT_LAUNCH_CHECK();
        }
        return VCT_OK;
    }
    if (!pos_sorted || !vol_sorted || !nl->col16 || !state64 || !u) return VCT_E_ARG;
    const int32_t* col_t = push_only ? nullptr : nl->col_t;
    if (dphi && !col_t && !nl->chunk_win) return VCT_E_ARG;   // the push form reads the stored windows
    if (dtheta && !proj) return VCT_E_ARG;
    const int64_t nnz = (dphi && col_t) ? nl->nnz : 0;   // the buffer is indexed by entries
    if (nnz < 0) return VCT_E_ARG;
    if (!ws || ws_bytes < vct_adjoint_workspace_size(dim, n, nnz, mp.nterms)) return VCT_E_WORKSPACE;
    Carver cv(ws, ws_bytes);
    const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
    double* partials = cv.take<double>((size_t)nred * (mp.nterms > 0 ? mp.nterms : 1));
    double* wbuf = cv.take<double>((size_t)(nnz > 0 ? nnz : 1));
    double* rowsum = cv.take<double>((size_t)n);
    double* partial = cv.take<double>((size_t)n * (dim == 3 ? 9 : 3));
    int32_t* wide = cv.take<int32_t>((size_t)(wide_list_len(n) + kWideList));
    const int64_t ncols = dim == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    AdjArgs a;
    a.n = n; a.invR = 1.0 / nl->R; a.g = g; a.pos = pos_sorted; a.vol = vol_sorted; a.state = state64; a.u = u;
    a.proj = proj; a.row_ptr = nl->row_ptr; a.col16 = nl->col16; a.col_t = col_t; a.cs = nl->cell_start;
    a.cstart = nl->chunk_start; a.cinfo = reinterpret_cast<const int4*>(nl->chunk_info);
    a.cwin = nl->chunk_win;
    a.nchunks = nl->chunk_off + ncols;
    a.chunk_off = nl->chunk_off;
    a.lap_row = group_row(dim, out_mask, VCT_OUT_LAP);
    if (pz) {
        const int r = group_row(dim, out_mask, VCT_OUT_PZ);
        a.r_gz = r, a.r_zz = r + 1, a.r_xz = r + 2, a.r_yz = dim == 3 ? r + 3 : -1;
    } else {   // PHESS component order: 3-D xx, yy, zz, xy, xz, yz; 2-D xx, zz, xz
        const int rg = group_row(dim, out_mask, VCT_OUT_PGRAD), rh = group_row(dim, out_mask, VCT_OUT_PHESS);
        a.r_gz = rg + dim - 1;
        a.r_zz = dim == 3 ? rh + 2 : rh + 1;
        a.r_xz = dim == 3 ? rh + 4 : rh + 2;
        a.r_yz = dim == 3 ? rh + 5 : -1;
    }
    a.nrows = n_out_rows(dim, out_mask);
    a.wbuf = wbuf; a.rowsum = rowsum; a.partial = partial; a.wide = wide; a.dphi = dphi;
    const int64_t cap = ncols + n / kChunk + 1;
    const bool overlap = !push_only;   // the allocation-free entry point makes no stream
    if (dim == 2)
        st = (kernel == VCT_KERNEL_WENDLAND_C2)
                 ? launch_adjoint<2, VCT_KERNEL_WENDLAND_C2>(a, cap, mp, dtheta, partials, overlap, s)
                 : launch_adjoint<2, VCT_KERNEL_CUBIC_SPLINE>(a, cap, mp, dtheta, partials, overlap, s);
    else
        st = (kernel == VCT_KERNEL_WENDLAND_C2)
                 ? launch_adjoint<3, VCT_KERNEL_WENDLAND_C2>(a, cap, mp, dtheta, partials, overlap, s)
                 : launch_adjoint<3, VCT_KERNEL_CUBIC_SPLINE>(a, cap, mp, dtheta, partials, overlap, s);
    return st;
}

extern "C" int vct_apply_ops_adjoint(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted,
                                     int kernel, const double* state64, uint32_t out_mask, const vct_map* map,
                                     const double* proj, const double* u, double* dphi, double* dtheta, void* ws,
                                     size_t ws_bytes, void* stream) {
    VCT_API_RANGE("vct_apply_ops_adjoint");
    return adjoint_run(nl, pos_sorted, vol_sorted, kernel, state64, out_mask, map, proj, u, dphi, dtheta, ws,
                       ws_bytes, false, stream);
}

// ------------------------------------------------------------------ reading R2 entry point

extern "C" size_t vct_adjoint_r2_workspace_size(int dim, int64_t n, int nterms) {
    if ((dim != 2 && dim != 3) || n < 0 || nterms < 0) return 0;
    const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
    const size_t n1 = (size_t)(n > 0 ? n : 1);
    const int ns = dim == 3 ? 9 : 3, npairs = dim == 3 ? 6 : 3;
    return aligned_sum({(size_t)(nred > 0 ? nred : 1) * (nterms > 0 ? nterms : 1) * 8, n1 * ns * sizeof(double),
                        n1 * npairs * sizeof(double), n1 * sizeof(double), n1 * sizeof(double),
                        (size_t)(wide_list_len(n) + kWideList) * 4});
}

extern "C" int vct_apply_ops_adjoint_r2(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted,
                                        int kernel, const double* state64, uint32_t out_mask, const vct_map* map,
                                        const double* proj, const double* phi, const double* u, double* dtheta,
                                        double* dzhat, void* ws, size_t ws_bytes, void* stream) {
    VCT_API_RANGE("vct_apply_ops_adjoint_r2");
    Grid g;
    int st = nlist_check(nl, g);
    if (st) return st;
    const int dim = nl->dim;
    const int64_t n = nl->n;
    const uint32_t need = VCT_OUT_LAP | VCT_OUT_PGRAD | VCT_OUT_PHESS;
    if (!map || !mask_valid(out_mask) || (out_mask & need) != need || (out_mask & VCT_OPT_GRAD1) ||
        (kernel != VCT_KERNEL_WENDLAND_C2 && kernel != VCT_KERNEL_CUBIC_SPLINE))
        return VCT_E_ARG;
    MapParams mp;
    st = map_params_from(map, dim, n, mp);
    if (st) return st;
    if (mp.kind == VCT_MAP_PER_PARTICLE) return VCT_E_ARG;   // the heights move with the bottom terms
    hipStream_t s = as_stream(stream);
    if (n == 0) {
        if (dtheta && mp.nterms > 0) {
            VCT_LAUNCH("k_zero_f64", k_zero_f64, dim3(1), dim3(64), 0, s, dtheta, (int64_t)mp.nterms);
            VCT_LAUNCH_CHECK();
        }
        return VCT_OK;
    }
    if (!pos_sorted || !vol_sorted || !state64 || !proj || !phi || !u || !nl->col16 || !nl->chunk_win)
        return VCT_E_ARG;
    if (!dtheta && !dzhat) return VCT_OK;
    if (!ws || ws_bytes < vct_adjoint_r2_workspace_size(dim, n, mp.nterms)) return VCT_E_WORKSPACE;
    Carver cv(ws, ws_bytes);
    const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
    double* partials = cv.take<double>((size_t)nred * (mp.nterms > 0 ? mp.nterms : 1));
    double* partial = cv.take<double>((size_t)n * (dim == 3 ? 9 : 3));
    double* r2h = cv.take<double>((size_t)n * (dim == 3 ? 6 : 3));
    double* r2b = cv.take<double>((size_t)n);
    double* gz = cv.take<double>((size_t)n);
    int32_t* wide = cv.take<int32_t>((size_t)(wide_list_len(n) + kWideList));
    const int64_t ncols = dim == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    AdjArgs a;
    memset(&a, 0, sizeof(a));
    a.n = n; a.invR = 1.0 / nl->R; a.g = g; a.pos = pos_sorted; a.vol = vol_sorted; a.state = state64; a.u = u;
    a.proj = proj; a.row_ptr = nl->row_ptr; a.col16 = nl->col16; a.cs = nl->cell_start;
    a.cstart = nl->chunk_start; a.cinfo = reinterpret_cast<const int4*>(nl->chunk_info);
    a.cwin = nl->chunk_win;
    a.nchunks = nl->chunk_off + ncols;
    a.chunk_off = nl->chunk_off;
    a.lap_row = group_row(dim, out_mask, VCT_OUT_LAP);
    const int rg = group_row(dim, out_mask, VCT_OUT_PGRAD), rh = group_row(dim, out_mask, VCT_OUT_PHESS);
    a.r_pg = rg;
    a.r_ph = rh;
    // PHESS component order: 3-D xx, yy, zz, xy, xz, yz; 2-D xx, zz, xz
    a.r_gz = rg + dim - 1;
    a.r_zz = dim == 3 ? rh + 2 : rh + 1;
    a.r_xz = dim == 3 ? rh + 4 : rh + 2;
    a.r_yz = dim == 3 ? rh + 5 : -1;
    a.nrows = n_out_rows(dim, out_mask);
    a.partial = partial; a.wide = wide; a.phi = phi; a.dzhat = dzhat;
    const int64_t cap = ncols + n / kChunk + 1;
    if (dim == 2)
        st = (kernel == VCT_KERNEL_WENDLAND_C2)
                 ? launch_r2<2, VCT_KERNEL_WENDLAND_C2>(a, cap, mp, gz, dtheta, partials, r2h, r2b, s)
                 : launch_r2<2, VCT_KERNEL_CUBIC_SPLINE>(a, cap, mp, gz, dtheta, partials, r2h, r2b, s);
    else
        st = (kernel == VCT_KERNEL_WENDLAND_C2)
                 ? launch_r2<3, VCT_KERNEL_WENDLAND_C2>(a, cap, mp, gz, dtheta, partials, r2h, r2b, s)
                 : launch_r2<3, VCT_KERNEL_CUBIC_SPLINE>(a, cap, mp, gz, dtheta, partials, r2h, r2b, s);
    return st;
}

// ------------------------------------------------------------------ allocation-free variant

// Scratch of vct_apply_ops_adjoint_noalloc.  Every GPU the library runs on
// holds its own copy until the process ends.  In host code the name `scratch`
// is a host-side stand-in, not a device address: host code only ever uses the
// address hipGetSymbolAddress returns on each device.
static __device__ __align__(256) unsigned char scratch[VCT_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// the current device's copy of `scratch`, looked up once per device
static int scratch_on_current_device(void** out) {
    int dev = -1;
    VCT_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return VCT_E_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        VCT_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return VCT_E_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return VCT_OK;
}

extern "C" int vct_apply_ops_adjoint_noalloc(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted,
                                             int kernel, const double* state64, uint32_t out_mask, const vct_map* map,
                                             const double* proj, const double* u, double* dphi, double* dtheta,
                                             void* stream) {
    VCT_API_RANGE("vct_apply_ops_adjoint_noalloc");
    if (!nl || (nl->dim != 2 && nl->dim != 3) || nl->n < 0 || !map || map->nterms < 0 ||
        map->nterms > VCT_MAX_TERMS)
        return VCT_E_ARG;
    // the push form's workspace (no entry buffer) must fit the scratch
    if (vct_adjoint_workspace_size(nl->dim, nl->n, 0, map->nterms) > (size_t)VCT_NOALLOC_SCRATCH_BYTES)
        return VCT_E_CAPACITY;
    void* ws = nullptr;
    const int st = scratch_on_current_device(&ws);
    if (st) return st;
    return adjoint_run(nl, pos_sorted, vol_sorted, kernel, state64, out_mask, map, proj, u, dphi, dtheta, ws,
                       (size_t)VCT_NOALLOC_SCRATCH_BYTES, true, stream);
}
