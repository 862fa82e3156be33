// Adjoint of the physical Laplacian operator (built on paper Eqs. lap_VCT and
// sec_SPH2; the adjoint itself is not in the paper).
//
// With lap_i = sum_{j in S_i} W_ij (phi_j - phi_i) and
//   W_ij = V_j c~_ij [P_a,i . r~_ij + (r~_ij' L~_i r~_ij) / |r~_ij|^4 P_s,i . q~_ij]
// (P_a,i, P_s,i the first- and second-order parts of particle i's Laplacian
// row of the state), the field cotangent is
//   dphi_k = sum_{i in S_k} u_i W_ik  -  sum_{j in S_k} u_k W_kj .
// Every particle i evaluates u_i W_ij once for its own row, with its own state
// in registers, and writes it at the transposed position col_t[e] (the entry
// (j, i) of row j) of a buffer, and its row sum to a second buffer; then every
// particle k sums its row of the first buffer in row order and subtracts its
// row sum.  No atomics, a fixed summation order, the same bits on every run.
//
// Bathymetry coefficients enter only through the VCT coefficients (projected
// positions are held fixed), so
//   dtheta_t = sum_i u_i (d c_trans_i / d coef_t) . D^ phi_i ,
// with d c_trans / d (h, h_x, h_y, h_xx, h_xy, h_yy) from forward-mode dual
// numbers, D^ phi_i from the projected-derivative rows of the forward apply,
// and d h^(k) / d coef_t the t-th term's basis products.  Per-particle
// contributions are reduced per work-group, then across work-groups, in a
// fixed order.
#include "common.h"
#include "map_dev.h"
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
    int lap_row, nrows;
    int r_gz, r_zz, r_xz, r_yz;   // rows of dz^, z^z^, x^z^, y^z^ (-1 in 2-D) in proj
    const double* coef;   // [n][kCoef] packed records of the gather form
    double* wbuf;      // [nnz]: u_i W_ij at the transposed position
    double* rowsum;    // [n]:  u_i sum_j W_ij
    double* dphi;
};

// Pass 1: u_i W_ij for every entry of row i, written transposed.  The first
// kALanes * kWSlots entries of each row (offset and transposed position) are
// loaded into registers up front; the window records are read from LDS one
// slot ahead of the arithmetic.
constexpr int kWSlots = 14;

template <int D, int KERNEL>
__device__ __forceinline__ double adj_weight(const double4& q, const double (&xi)[3], double invR,
                                             const double (&L2)[Dims<D>::nL], const double (&Pl)[Dims<D>::nk]) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, m = Dm::m;
    double r[D];
    r[0] = (q.x - xi[0]) * invR;
    r[1] = (q.y - xi[1]) * invR;
    if (D == 3) r[D - 1] = (q.z - xi[2]) * invR;
    double q2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) q2 += r[a] * r[a];
    double qv[m];
#pragma unroll
    for (int p = 0; p < m; ++p) qv[p] = r[pair_a<D>(p)] * r[pair_b<D>(p)];
    double rLr = 0.0, sa = 0.0, ss = 0.0;
#pragma unroll
    for (int p = 0; p < nL; ++p) rLr += L2[p] * qv[p];
#pragma unroll
    for (int a = 0; a < D; ++a) sa += Pl[a] * r[a];
#pragma unroll
    for (int p = 0; p < m; ++p) ss += Pl[D + p] * qv[p];
    const double vc = q.w * kernel_shape<KERNEL>(vsqrt(q2));
    return vc * (sa + rLr * vrcp(q2 * q2) * ss);
}

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
    auto cols = [&](int s) -> int { return (int)((cpk[s / 2] >> (16 * (s % 2))) & 0xffffu); };
    __syncthreads();
    const int W = __builtin_amdgcn_readfirstlane(w.off[w.nr]);
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
                const double wij = adj_weight<D, KERNEL>(q, xi, A.invR, L2, Pl);
                A.wbuf[tcol[s]] = wij;
                sum += wij;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
#pragma unroll 1
        for (int s = 0; s < kWSlots; ++s) {
            if (s < nslot) {
                const double wij = adj_weight<D, KERNEL>(fetch(cols(s)), xi, A.invR, L2, Pl);
                A.wbuf[tcol[s]] = wij;
                sum += wij;
            }
        }
    }
    for (int64_t e = rb + lane + (int64_t)kALanes * kWSlots; e < re; e += kALanes) {
        const double wij = adj_weight<D, KERNEL>(fetch(A.col16[e]), xi, A.invR, L2, Pl);
        A.wbuf[A.col_t[e]] = wij;
        sum += wij;
    }
    sum = group_sum(sum, kALanes);
    if (valid && lane == 0) A.rowsum[ii] = sum;
}

// Gather form (no transposed map): per particle, [L~ (nL, off-diagonals
// doubled), u P_lap (d + m), 0...] packed in one 128-byte record, so the
// rebuild of W_ik from row i reads a single cache line per neighbour.
constexpr int kCoef = 16;
template <int D>
__global__ __launch_bounds__(256) void k_adjoint_pack(int64_t n, const double* __restrict__ state, int lap_row,
                                                      const double* __restrict__ u, double* __restrict__ coef) {
    using Dm = Dims<D>;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double c[kCoef];
#pragma unroll
    for (int k = 0; k < kCoef; ++k) c[k] = 0.0;
#pragma unroll
    for (int p = 0; p < Dm::nL; ++p)
        c[p] = (pair_a<D>(p) == pair_b<D>(p) ? 1.0 : 2.0) * state[(int64_t)p * n + i];
    const double ui = u[i];
#pragma unroll
    for (int k = 0; k < Dm::nk; ++k) c[Dm::nL + k] = ui * state[(int64_t)(Dm::nL + lap_row * Dm::nk + k) * n + i];
    double2* dst = reinterpret_cast<double2*>(coef + i * kCoef);
#pragma unroll
    for (int k = 0; k < kCoef / 2; ++k) dst[k] = make_double2(c[2 * k], c[2 * k + 1]);
}

// dphi_k = sum_{i in S_k} u_i W_ik - u_k sum_j W_kj, both over the row of k.
// The chunk's window is walked in sub-windows of kASub particles whose
// records (position, volume and the packed 128-byte record) are staged in
// LDS; a row's offsets ascend, so every lane keeps a cursor into its strided
// share of the row and consumes the entries that fall in the current
// sub-window.
// A record is 11 16-byte slots (176 B = 44 banks of 4 B, an odd multiple of
// 16 B): the lanes reading 16 consecutive records in one LDS pass start on 16
// different bank quadruples, where a 160-byte record would give 8.
#ifndef VCT_ASUB
#define VCT_ASUB 448
#endif
#ifndef VCT_DPHI_GROUPS
#define VCT_DPHI_GROUPS 2
#endif
constexpr int kASub = VCT_ASUB;   // records per sub-window: 448 x 176 B, two groups per CU

template <int D, int KERNEL>
__global__ __launch_bounds__(kAThreads, VCT_DPHI_GROUPS) void k_adjoint_dphi(AdjArgs A) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, nk = Dm::nk, m = Dm::m;
    constexpr int kRec = 11;   // double2 per record: (x, y), (z, V), the packed record, one pad
    __shared__ double2 srec[kASub * kRec];
    __shared__ WindowT<D> w;
    __shared__ double sx[kChunk];
    __shared__ int sord[kChunk];
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *A.nchunks) return;   // uniform over the work-group
    const int64_t n = A.n;
    const int64_t p0 = A.cstart[b], p1 = A.cstart[b + 1];
    const int np = (int)(p1 - p0);
    if (threadIdx.x < kWave) {
        if (A.cwin) window_load<D>(A.cwin, b, w);
        else chunk_window_wave<D>(A.g, A.cs, A.cinfo[b], w);
    } else if (threadIdx.x < 2 * kWave) {
        const int q = threadIdx.x - kWave;
        if (q < np) sx[q] = A.pos[p0 + q];
    }
    __syncthreads();
    // The waves take the chunk's particles in order of x: a sub-window holds
    // about one x-layer of the window's columns, so particles with close x
    // have similar shares of their rows in it, and the cursor loops of a wave
    // end together (ties by index).
    if (threadIdx.x < kChunk && (int)threadIdx.x < np) {
        const int q = threadIdx.x;
        const double xq = sx[q];
        int r = 0;
        for (int j = 0; j < np; ++j) {
            const double xj = sx[j];
            r += (xj < xq || (xj == xq && j < q)) ? 1 : 0;
        }
        sord[r] = q;
    }
    __syncthreads();
    const int lane = threadIdx.x % kALanes;
    const int slot = threadIdx.x / kALanes;
    const bool valid = slot < np;
    const int64_t k = p0 + (valid ? sord[slot] : 0);
    const int64_t kk = valid ? k : p0;
    double xk[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xk[a] = a < D ? A.pos[a * n + kk] : 0.0;
    const double* ck = A.coef + kk * kCoef;
    double Lk2[nL], Pk[nk];
#pragma unroll
    for (int p = 0; p < nL; ++p) Lk2[p] = ck[p];
#pragma unroll
    for (int c = 0; c < nk; ++c) Pk[c] = ck[nL + c];   // u_k P_lap,k
    const double Vk = A.vol[kk];
    const int64_t re = valid ? A.row_ptr[kk + 1] : 0;
    int64_t e = (valid ? A.row_ptr[kk] : 0) + lane;
    int tn = e < re ? (int)A.col16[e] : INT_MAX;
    const int W = __builtin_amdgcn_readfirstlane(w.off[w.nr]);
    double acc1 = 0.0, self = 0.0;
    for (int s0 = 0; s0 < W; s0 += kASub) {
        const int s1 = W - s0 < kASub ? W : s0 + kASub;
        if (s0 > 0) __syncthreads();   // the previous sub-window is consumed
        for (int t = s0 + (int)threadIdx.x; t < s1; t += kAThreads) {
            const int64_t j = window_global<D>(w, t);
            double2* dst = srec + (t - s0) * kRec;
            dst[0] = make_double2(A.pos[j], A.pos[n + j]);
            dst[1] = make_double2(D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
            const double2* src = reinterpret_cast<const double2*>(A.coef + j * kCoef);
#pragma unroll
            for (int c = 0; c < kCoef / 2; ++c) dst[2 + c] = src[c];
        }
        __syncthreads();
        while (tn < s1) {
            const double2* rec = srec + (tn - s0) * kRec;
            e += kALanes;
            tn = e < re ? (int)A.col16[e] : INT_MAX;
            const double2 qa = rec[0], qb = rec[1];
            const double4 q = make_double4(qa.x, qa.y, qb.x, qb.y);
            double ci[kCoef];
#pragma unroll
            for (int c = 0; c < kCoef / 2; ++c) {
                const double2 v = rec[2 + c];
                ci[2 * c] = v.x;
                ci[2 * c + 1] = v.y;
            }
            double r[D];   // r~_ki
            r[0] = (q.x - xk[0]) * A.invR;
            r[1] = (q.y - xk[1]) * A.invR;
            if (D == 3) r[D - 1] = (q.z - xk[2]) * A.invR;
            double q2 = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) q2 += r[a] * r[a];
            double qv[m];
#pragma unroll
            for (int p = 0; p < m; ++p) qv[p] = r[pair_a<D>(p)] * r[pair_b<D>(p)];
            const double c = kernel_shape<KERNEL>(vsqrt(q2));
            const double iq4 = vrcp(q2 * q2);
            double rLk = 0.0, rLi = 0.0, sak = 0.0, ssk = 0.0, sai = 0.0, ssi = 0.0;
#pragma unroll
            for (int p = 0; p < nL; ++p) {
                rLk += Lk2[p] * qv[p];
                rLi += ci[p] * qv[p];
            }
#pragma unroll
            for (int a = 0; a < D; ++a) {
                sak += Pk[a] * r[a];
                sai += ci[nL + a] * r[a];
            }
#pragma unroll
            for (int p = 0; p < m; ++p) {
                ssk += Pk[D + p] * qv[p];
                ssi += ci[nL + D + p] * qv[p];
            }
            // u_k W_ki (row k: volume V_i, correction of k) and u_i W_ik (row i:
            // r~_ik = -r~_ki, volume V_k, correction of i)
            self += q.w * c * (sak + rLk * iq4 * ssk);
            acc1 += Vk * c * (rLi * iq4 * ssi - sai);
        }
    }
    acc1 = group_sum(acc1, kALanes);
    self = group_sum(self, kALanes);
    if (valid && lane == 0) A.dphi[kk] = acc1 - self;
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
template <int D>
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

template <int D, int KERNEL>
static int launch_adjoint(AdjArgs a, int64_t cap, const MapParams& mp, double* dtheta, double* partials,
                          hipStream_t s) {
    const int64_t n = a.n;
    if (a.dphi && a.col_t) {
        VCT_LAUNCH("k_adjoint_weights", (k_adjoint_weights<D, KERNEL>), dim3((unsigned)cap), dim3(kAThreads), 0, s, a);
        VCT_LAUNCH_CHECK();
        VCT_LAUNCH("k_adjoint_gather", k_adjoint_gather, dim3((unsigned)((n * kALanes + 255) / 256)), dim3(256), 0,
                   s, n, a.row_ptr, a.wbuf, a.rowsum, a.dphi);
        VCT_LAUNCH_CHECK();
    } else if (a.dphi) {
        VCT_LAUNCH("k_adjoint_pack", (k_adjoint_pack<D>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                   a.state, a.lap_row, a.u, const_cast<double*>(a.coef));
        VCT_LAUNCH_CHECK();
        VCT_LAUNCH("k_adjoint_dphi", (k_adjoint_dphi<D, KERNEL>), dim3((unsigned)cap), dim3(kAThreads), 0, s, a);
        VCT_LAUNCH_CHECK();
    }
    if (dtheta && mp.nterms > 0) {
        const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
        VCT_LAUNCH("k_dtheta_partials", (k_dtheta_partials<D>), dim3((unsigned)nred), dim3(kRedThreads), 0, s, a,
                   mp, partials);
        VCT_LAUNCH_CHECK();
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

}  // namespace vct

using namespace vct;

extern "C" size_t vct_adjoint_workspace_size(int dim, int64_t n, int64_t nnz, int nterms) {
    if ((dim != 2 && dim != 3) || n < 0 || nnz < 0 || nterms < 0) return 0;
    const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
    return aligned_sum({(size_t)(nred > 0 ? nred : 1) * (nterms > 0 ? nterms : 1) * 8,
                        (size_t)(nnz > 0 ? nnz : 1) * sizeof(double), (size_t)(n > 0 ? n : 1) * sizeof(double),
                        (size_t)(n > 0 ? n : 1) * kCoef * sizeof(double)});
}

extern "C" int vct_apply_ops_adjoint(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted,
                                     int kernel, const double* state64, uint32_t out_mask, const vct_map* map,
                                     const double* proj, const double* u, double* dphi, double* dtheta, void* ws,
                                     size_t ws_bytes, void* stream) {
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
    st = map_params_from(map, dim, mp);
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
    if (dtheta && !proj) return VCT_E_ARG;
    const int64_t nnz = (dphi && nl->col_t) ? nl->nnz : 0;   // the buffer is indexed by entries
    if (nnz < 0) return VCT_E_ARG;
    if (!ws || ws_bytes < vct_adjoint_workspace_size(dim, n, nnz, mp.nterms)) return VCT_E_WORKSPACE;
    Carver cv(ws, ws_bytes);
    const int64_t nred = (n + kRedThreads - 1) / kRedThreads;
    double* partials = cv.take<double>((size_t)nred * (mp.nterms > 0 ? mp.nterms : 1));
    double* wbuf = cv.take<double>((size_t)(nnz > 0 ? nnz : 1));
    double* rowsum = cv.take<double>((size_t)n);
    double* coef = cv.take<double>((size_t)n * kCoef);
    const int64_t ncols = dim == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    AdjArgs a;
    a.n = n; a.invR = 1.0 / nl->R; a.g = g; a.pos = pos_sorted; a.vol = vol_sorted; a.state = state64; a.u = u;
    a.proj = proj; a.row_ptr = nl->row_ptr; a.col16 = nl->col16; a.col_t = nl->col_t; a.cs = nl->cell_start;
    a.cstart = nl->chunk_start; a.cinfo = reinterpret_cast<const int4*>(nl->chunk_info);
    a.cwin = nl->chunk_win;
    a.nchunks = nl->chunk_off + ncols;
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
    a.wbuf = wbuf; a.rowsum = rowsum; a.coef = coef; a.dphi = dphi;
    const int64_t cap = ncols + n / kChunk + 1;
    if (dim == 2)
        st = (kernel == VCT_KERNEL_WENDLAND_C2)
                 ? launch_adjoint<2, VCT_KERNEL_WENDLAND_C2>(a, cap, mp, dtheta, partials, s)
                 : launch_adjoint<2, VCT_KERNEL_CUBIC_SPLINE>(a, cap, mp, dtheta, partials, s);
    else
        st = (kernel == VCT_KERNEL_WENDLAND_C2)
                 ? launch_adjoint<3, VCT_KERNEL_WENDLAND_C2>(a, cap, mp, dtheta, partials, s)
                 : launch_adjoint<3, VCT_KERNEL_CUBIC_SPLINE>(a, cap, mp, dtheta, partials, s);
    return st;
}
