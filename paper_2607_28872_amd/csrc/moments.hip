// Moment assembly and per-particle solve, FP64 (paper Sec. 3.1, Eqs. gra_1st
// and sec_SPH2), folded with the VCT coefficients (Sec. 2.1).
//
// Formulation.  With r~ = r_ij / R, c~ the kernel shape (grad w = K c~ r~) and
// q~ the quadratic monomials of r~, expanding phi_ij to second order and taking
// moments against V c~ r~ (d rows) and V F~ q~ (m rows) gives the block system
//     [ A  B ] [ R grad phi ]   [ a ]    A = sum V c~ r~ r~^T   B = sum V c~ r~ q~^T
//     [ C  E ] [ R^2 D / 2  ] = [ s ]    C = sum V F~ q~ r~^T   E = sum V F~ q~ q~^T
// with F~ = c~ (r~^T L r~) / |r~|^4, L = A^-1 (the paper's first-order
// correction, F_ij of Eq. sec_SPH2 up to constant factors), a = sum V c~ phi_ij r~,
// s = sum V F~ q~ phi_ij.  Eliminating the first block row reproduces Eq.
// sec_SPH2: M = E - C L B and D/2 = M^-1 (s - C L a), and the second-order
// gradient is L a - (L B) D/2.  Only the distinct monomials are accumulated
// (3rd and 4th order: 10 and 15 in 3-D); the two sweeps differ because F~
// needs L from the first.
//
// Kernel 1 (one group of G lanes per particle) runs the sweeps and writes the
// monomial sums.  Kernel 2 (one thread per particle) solves the Schur system
// with partial pivoting and writes, per output row o and neighbour sum c, the
// coefficient P_i[o][c] of the physical output in terms of [a; s].
#include <type_traits>

#include "common.h"
#include "map_dev.h"
#include "tiles.h"

namespace vct {

template <int D> struct MomLayout {
    static constexpr int nL = Dims<D>::nL, n3 = Dims<D>::n3, n4 = Dims<D>::n4;
    static constexpr int oL = 0, oB = nL, oC = nL + n3, oE = nL + 2 * n3;
    static constexpr int total = nL + 2 * n3 + n4;
};

constexpr double kPivotTol = 1e-12;

// inverse of a symmetric d x d matrix (pairs order), false if singular
template <int D>
__device__ __forceinline__ bool sym_inverse(const double (&A)[Dims<D>::nL], double (&L)[Dims<D>::nL]) {
    if (D == 2) {
        // pairs [xx, zz, xz]
        double a = A[0], c = A[1], b = A[2];
        double det = a * c - b * b;
        double sc = fmax(fabs(a), fmax(fabs(b), fabs(c)));
        bool bad = !(fabs(det) > kPivotTol * sc * sc) || !isfinite(det);
        double id = 1.0 / det;
        L[0] = c * id; L[1] = a * id; L[2] = -b * id;
        return !bad;
    } else {
        // pairs [xx, yy, zz, xy, xz, yz]
        double a00 = A[0], a11 = A[1], a22 = A[2], a01 = A[3], a02 = A[4], a12 = A[5];
        double c00 = a11 * a22 - a12 * a12;
        double c01 = a02 * a12 - a01 * a22;
        double c02 = a01 * a12 - a02 * a11;
        double c11 = a00 * a22 - a02 * a02;
        double c12 = a01 * a02 - a00 * a12;
        double c22 = a00 * a11 - a01 * a01;
        double det = a00 * c00 + a01 * c01 + a02 * c02;
        double sc = 0.0;
        for (int k = 0; k < 6; ++k) sc = fmax(sc, fabs(A[k]));
        bool bad = !(fabs(det) > kPivotTol * sc * sc * sc) || !isfinite(det);
        double id = 1.0 / det;
        L[0] = c00 * id; L[1] = c11 * id; L[2] = c22 * id;
        L[3] = c01 * id; L[4] = c02 * id; L[5] = c12 * id;
        return !bad;
    }
}

template <int D>
__device__ __forceinline__ double sym_at(const double (&S)[Dims<D>::nL], int a, int b) {
    // element (a, b) of a symmetric matrix stored in pairs order
    if (D == 2) return (a == b) ? S[a] : S[2];
    if (a == b) return S[a];
    int lo = a < b ? a : b, hi = a < b ? b : a;
    return (lo == 0 && hi == 1) ? S[3] : (lo == 0 ? S[4] : S[5]);
}

// ------------------------------------------------------------------ kernel 1: sweeps

// Launch shape (overridable at build time for tuning).  A work-group is one
// chunk with kMLanes lanes per particle; its LDS (window records plus the L
// and B sums of the chunk, about 53 KB at 1400 records) and its registers (at
// most 168 VGPRs) let three work-groups share a CU, so the staging of one
// overlaps the sweeps of the others.  Windows larger than kMWin (about 1% at
// the 8.4M-particle sigma set) read their records from global memory.
#ifndef VCT_MLANES
#define VCT_MLANES 4
#endif
#ifndef VCT_MWIN
#define VCT_MWIN 1400
#endif
#ifndef VCT_SWEEP_WAVES
#define VCT_SWEEP_WAVES 3
#endif
#ifndef VCT_MSLOTS
#define VCT_MSLOTS 28
#endif
#ifndef VCT_SWEEP2_AHEAD
#define VCT_SWEEP2_AHEAD true
#endif
constexpr int kMLanes = VCT_MLANES;           // lanes per particle
constexpr int kMThreads = kChunk * kMLanes;   // one chunk per work-group
constexpr int kMWin = VCT_MWIN;               // LDS window capacity (records)
constexpr int kMSlots = VCT_MSLOTS;           // row entries per lane held in registers

struct SweepArgs {
    int64_t n;
    double invR;
    Grid g;
    const double* pos;
    const double* vol;
    const int64_t* row_ptr;
    const uint16_t* col16;
    const int64_t* cs;
    const int32_t* cstart;
    const int4* cinfo;
    const int32_t* cwin;   // stored windows or NULL
    const int64_t* nchunks;
    double* mom;
    uint8_t* mflags;
};

// One chunk per work-group: the window's positions and volumes are staged in
// LDS (x, y, z, V per record), kMLanes lanes per particle hold their share of
// the row's window offsets in registers and read the records from LDS one
// entry ahead of the arithmetic, for both sweeps; the sums are reduced across
// the group and written through LDS with unit stride.
template <int D, int KERNEL>
__global__ __launch_bounds__(kMThreads, VCT_SWEEP_WAVES) void k_moment_sweeps(SweepArgs A) {
    using Dm = Dims<D>;
    using ML = MomLayout<D>;
    __shared__ double4 sd[kMWin];
    __shared__ double sLB[ML::oC * kChunk];   // L and B of every particle, kept out of registers in sweep 2
    __shared__ WindowT<D> w;
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *A.nchunks) return;   // uniform over the work-group
    const int64_t n = A.n;
    const int64_t p0 = A.cstart[b], p1 = A.cstart[b + 1];
    if (threadIdx.x < kWave) {
        if (A.cwin) window_load<D>(A.cwin, b, w);
        else chunk_window_wave<D>(A.g, A.cs, A.cinfo[b], w);
    }
    const int lane = threadIdx.x % kMLanes;
    const int pl = threadIdx.x / kMLanes;
    const int64_t i = p0 + pl;
    const bool valid = i < p1;
    const int64_t ii = valid ? i : p0;
    double xi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xi[a] = a < D ? A.pos[a * n + ii] : 0.0;
    const double Vi = A.vol[ii];
    const int64_t rb = valid ? A.row_ptr[ii] : 0, re = valid ? A.row_ptr[ii + 1] : 0;
    uint32_t cpk[(kMSlots + 1) / 2];
    int nslot = 0;
    {
        const uint32_t first = re > rb ? (uint32_t)A.col16[rb] : 0u;
        const int len = (int)(re - rb);        // 32-bit row-local indices: one base address,
        const uint16_t* crow = A.col16 + rb + lane;   // immediate offsets per slot
#pragma unroll
        for (int s = 0; s < kMSlots; ++s) {
            const bool in = lane + kMLanes * s < len;
            const uint32_t c = in ? (uint32_t)crow[kMLanes * s] : first;
            nslot += in ? 1 : 0;
            if (s % 2 == 0) cpk[s / 2] = c;
            else cpk[s / 2] |= c << 16;
        }
    }
    __syncthreads();
    const int W = __builtin_amdgcn_readfirstlane(w.off[w.nr]);
    auto cols = [&](int s) -> int { return dcheck((int)((cpk[s / 2] >> (16 * (s % 2))) & 0xffffu), W, kChkWindow); };
    const bool in_lds = W <= kMWin;
    if (in_lds) {
        // every load of a thread is issued before its first LDS store
        constexpr int kRep = (kMWin + kMThreads - 1) / kMThreads;
        double4 q[kRep];
#pragma unroll
        for (int k = 0; k < kRep; ++k) {
            const int t = threadIdx.x + k * kMThreads;
            if (t < W) {   // lanes past the window load nothing (whole waves skip)
                const int64_t j = window_global<D>(w, t);
                q[k] = make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
            }
        }
#pragma unroll
        for (int k = 0; k < kRep; ++k) {
            const int t = threadIdx.x + k * kMThreads;
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
    // The offsets r = r^_j - r^_i and their pair products q, unscaled (q
    // holds the squares first, so |r|^2 is their sum): every sum below is a
    // homogeneous polynomial in r, so the scaling by 1/R of the moment
    // formulation (r~ = r / R) is applied once to each total instead of to
    // every offset -- A~ = A / R^2, B~ = B / R^3, C~ = C / R, E~ = E / R^2 (in
    // sweep 2 the weight V F~ = V c~ (r~' L~ r~) / |r~|^4 equals R^2 times
    // V c~ (r' L~ r) / |r|^4).
    auto geom = [&](const double4& q, double (&r)[D], double (&qv)[Dm::m], double& q2) {
        r[0] = q.x - xi[0];
        r[1] = q.y - xi[1];
        if (D == 3) r[D - 1] = q.z - xi[2];
#pragma unroll
        for (int p = 0; p < Dm::m; ++p) qv[p] = r[pair_a<D>(p)] * r[pair_b<D>(p)];
        q2 = qv[0];
#pragma unroll
        for (int a = 1; a < D; ++a) q2 += qv[a];
    };
    // visits every row entry: the register slots (records read one ahead
    // when the window is in LDS), then the rest of a long row
    auto sweep = [&](auto&& body, auto ahead) {
        if (in_lds && decltype(ahead)::value) {
            double4 qn = sd[cols(0)];
#pragma unroll
            for (int s = 0; s < kMSlots; ++s) {
                const double4 q = qn;
                if (s + 1 < kMSlots) qn = sd[cols(s + 1)];
                __builtin_amdgcn_sched_barrier(0);
                if (s < nslot) body(q);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else if (in_lds) {
#pragma unroll
            for (int s = 0; s < kMSlots; ++s)
                if (s < nslot) body(sd[cols(s)]);
        } else {
#pragma unroll 1
            for (int s = 0; s < kMSlots; ++s)
                if (s < nslot) body(fetch(cols(s)));
        }
        for (int64_t e = rb + lane + (int64_t)kMLanes * kMSlots; e < re; e += kMLanes) body(fetch(A.col16[e]));
    };
    int fl = 0;
    if (valid && re - rb < D + Dm::m) fl |= VCT_FLAG_FEW;
    bool fin = isfinite(Vi);
#pragma unroll
    for (int a = 0; a < D; ++a) fin = fin && isfinite(xi[a]);
    if (!fin) fl |= VCT_FLAG_NONFINITE;

    // sweep 1: A (pairs) and B (3rd-order monomials), weights V c~
    double Am[Dm::nL], B[Dm::n3];
#pragma unroll
    for (int p = 0; p < Dm::nL; ++p) Am[p] = 0.0;
#pragma unroll
    for (int t = 0; t < Dm::n3; ++t) B[t] = 0.0;
    // The weighted offsets wr = wgt r~ are formed once per pair; the pair and
    // cubic sums are then one multiply-add each (wr times r~ or q~), not a
    // monomial product followed by a weighted multiply-add.
    double q2min = 1.0;   // a zero offset marks a duplicate (tested after the sweep)
    sweep([&](const double4& q) {
        double r[D], q2, qv[Dm::m], wr[D];
        geom(q, r, qv, q2);
        q2min = fmin(q2min, q2);
        const double wgt = q.w * kernel_shape<KERNEL>(vsqrt(q2) * A.invR);
#pragma unroll
        for (int a = 0; a < D; ++a) wr[a] = wgt * r[a];
#pragma unroll
        for (int p = 0; p < Dm::nL; ++p) Am[p] += wr[pair_a<D>(p)] * r[pair_b<D>(p)];
#pragma unroll
        for (int t = 0; t < Dm::n3; ++t)
            B[t] += wr[mono_comp<D, 3>(t, 0)] * qv[sym_index<D>(mono_comp<D, 3>(t, 1), mono_comp<D, 3>(t, 2))];
    }, std::true_type{});
    if (q2min == 0.0) fl |= VCT_FLAG_DUPLICATE;
    const double invR2 = A.invR * A.invR;
#pragma unroll
    for (int p = 0; p < Dm::nL; ++p) Am[p] = group_sum(Am[p], kMLanes) * invR2;
#pragma unroll
    for (int t = 0; t < Dm::n3; ++t) B[t] = group_sum(B[t], kMLanes) * (invR2 * A.invR);
    // a non-finite neighbour position or volume makes some sum non-finite
    // (every weight is positive), which is cheaper to test once than per pair
    {
        bool sf = true;
#pragma unroll
        for (int p = 0; p < Dm::nL; ++p) sf = sf && isfinite(Am[p]);
#pragma unroll
        for (int t = 0; t < Dm::n3; ++t) sf = sf && isfinite(B[t]);
        if (!sf) fl |= VCT_FLAG_NONFINITE;
    }
    for (int m_ = kMLanes >> 1; m_ >= 1; m_ >>= 1) fl |= __shfl_xor(fl, m_, kWave);

    double L[Dm::nL];
    if (!sym_inverse<D>(Am, L)) fl |= VCT_FLAG_SINGULAR_A;
    double L2[Dm::nL];
#pragma unroll
    for (int p = 0; p < Dm::nL; ++p) L2[p] = (pair_a<D>(p) == pair_b<D>(p) ? 1.0 : 2.0) * L[p];
#pragma unroll
    for (int v = 0; v < ML::oC; ++v)
        if (v % kMLanes == lane) sLB[v * kChunk + pl] = v < ML::oB ? L[v] : B[v - ML::oB];

    // sweep 2: C (3rd order) and E (4th order), weights V F~ (skipped for a
    // flagged particle: its state is NaN anyway)
    double Cm[Dm::n3], E[Dm::n4];
#pragma unroll
    for (int t = 0; t < Dm::n3; ++t) Cm[t] = 0.0;
#pragma unroll
    for (int t = 0; t < Dm::n4; ++t) E[t] = 0.0;
    const bool live = fl == 0;
    sweep([&](const double4& q) {
        double r[D], q2, qv[Dm::m], wq[Dm::m];
        geom(q, r, qv, q2);
        double rLr = 0.0;
#pragma unroll
        for (int p = 0; p < Dm::nL; ++p) rLr += L2[p] * qv[p];
        // |r| = q2 / sqrt(q2) and 1/|r|^4 = (1/sqrt(q2))^4 from one refined reciprocal square root
        const double y = vrsq(q2), y2 = y * y;
        const double wgt = live ? q.w * kernel_shape<KERNEL>(q2 * y * A.invR) * rLr * (y2 * y2) : 0.0;
#pragma unroll
        for (int p = 0; p < Dm::m; ++p) wq[p] = wgt * qv[p];
#pragma unroll
        for (int t = 0; t < Dm::n3; ++t)
            Cm[t] += wq[sym_index<D>(mono_comp<D, 3>(t, 0), mono_comp<D, 3>(t, 1))] * r[mono_comp<D, 3>(t, 2)];
#pragma unroll
        for (int t = 0; t < Dm::n4; ++t)
            E[t] += wq[sym_index<D>(mono_comp<D, 4>(t, 0), mono_comp<D, 4>(t, 1))] *
                    qv[sym_index<D>(mono_comp<D, 4>(t, 2), mono_comp<D, 4>(t, 3))];
    }, std::integral_constant<bool, VCT_SWEEP2_AHEAD>{});
#pragma unroll
    for (int t = 0; t < Dm::n3; ++t) Cm[t] = group_sum(Cm[t], kMLanes) * A.invR;
#pragma unroll
    for (int t = 0; t < Dm::n4; ++t) E[t] = group_sum(E[t], kMLanes) * invR2;

    // the sums through LDS (the window is no longer needed), then unit-stride
    // stores: thread t writes entries (v, q) with q = t % kChunk
    static_assert(ML::total * kChunk * 8 <= kMWin * 32, "sum staging must fit the window buffer");
    double* ssum = reinterpret_cast<double*>(sd);
    __syncthreads();
#pragma unroll
    for (int v = ML::oC; v < ML::total; ++v) {
        if (v % kMLanes != lane) continue;
        ssum[(v - ML::oC) * kChunk + pl] = v < ML::oE ? Cm[v - ML::oC] : E[v - ML::oE];
    }
    __syncthreads();
    {
        const int q = threadIdx.x % kChunk;
        if (p0 + q < p1)
            for (int v = threadIdx.x / kChunk; v < ML::total; v += kMThreads / kChunk)
                A.mom[(int64_t)v * n + p0 + q] = v < ML::oC ? sLB[v * kChunk + q] : ssum[(v - ML::oC) * kChunk + q];
    }
    if (valid && lane == 0) A.mflags[ii] = (uint8_t)fl;
}

// ------------------------------------------------------------------ kernel 2: solve + fold

// In-place inverse by Gauss-Jordan elimination with partial (row) pivoting;
// false if a pivot falls below kPivotTol times the largest entry.  One
// division per pivot; the row interchanges become column interchanges of the
// inverse, undone at the end.
template <int M>
__device__ __forceinline__ bool gj_invert(double (&A)[M][M]) {
    double scale = 0.0;
#pragma unroll
    for (int r = 0; r < M; ++r)
#pragma unroll
        for (int c = 0; c < M; ++c) scale = fmax(scale, fabs(A[r][c]));
    bool bad = !(scale > 0.0) || !isfinite(scale);
    int piv[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        int p = c;
        double best = fabs(A[c][c]);
#pragma unroll
        for (int r = c + 1; r < M; ++r) {
            const double v = fabs(A[r][c]);
            if (v > best) { best = v; p = r; }
        }
        piv[c] = p;
        if (!(best > kPivotTol * scale)) bad = true;
#pragma unroll
        for (int r = c + 1; r < M; ++r) {
            if (r == p) {
#pragma unroll
                for (int k = 0; k < M; ++k) { const double t = A[c][k]; A[c][k] = A[r][k]; A[r][k] = t; }
            }
        }
        const double inv = 1.0 / A[c][c];
        A[c][c] = 1.0;
#pragma unroll
        for (int k = 0; k < M; ++k) A[c][k] *= inv;
#pragma unroll
        for (int r = 0; r < M; ++r) {
            if (r == c) continue;
            const double f = A[r][c];
            A[r][c] = 0.0;
#pragma unroll
            for (int k = 0; k < M; ++k) A[r][k] -= f * A[c][k];
        }
    }
#pragma unroll
    for (int c = M - 1; c >= 0; --c) {
#pragma unroll
        for (int r = c + 1; r < M; ++r) {
            if (r == piv[c]) {
#pragma unroll
                for (int k = 0; k < M; ++k) { const double t = A[k][c]; A[k][c] = A[k][r]; A[k][r] = t; }
            }
        }
    }
    return !bad;
}

#ifndef VCT_SOLVE_WAVES
#define VCT_SOLVE_WAVES 2
#endif
// One folded state: its output rows and where it goes (either array may be null).
struct SolveOut {
    uint32_t mask;
    int nrows;
    double* s64;
    float* s32;
};

// TWO: a second state with other output rows folded from the same inverse
// (the map and the VCT_OPT_GRAD1 choice are shared).
template <int D, bool TWO>
__global__ __launch_bounds__(128, VCT_SOLVE_WAVES) void k_moment_solve(int64_t n, const double* __restrict__ pos,
                                                      const double* __restrict__ mom,
                                                      const uint8_t* __restrict__ mflags, double invR,
                                                      MapParams mp, SolveOut o1, SolveOut o2,
                                                      uint8_t* __restrict__ flags_out,
                                                      unsigned long long* __restrict__ nflag) {
    using Dm = Dims<D>;
    using ML = MomLayout<D>;
    constexpr int d = D, m = Dm::m, nL = Dm::nL, nk = Dm::nk;
    const int64_t i = (int64_t)xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int fl = mflags[i];
    double L[nL];
    for (int p = 0; p < nL; ++p) L[p] = mom[(int64_t)(ML::oL + p) * n + i];

    // B~ (d x m), C~ (m x d), E~ (m x m) from the distinct monomial sums
    double Bt[d][m], Ct[m][d], M[m][m];
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
        for (int p = 0; p < m; ++p) {
            Bt[a][p] = mom[(int64_t)(ML::oB + mono3_index<D>(a, pair_a<D>(p), pair_b<D>(p))) * n + i];
            Ct[p][a] = mom[(int64_t)(ML::oC + mono3_index<D>(pair_a<D>(p), pair_b<D>(p), a)) * n + i];
        }
#pragma unroll
    for (int p = 0; p < m; ++p)
#pragma unroll
        for (int q = 0; q < m; ++q)
            M[p][q] = mom[(int64_t)(ML::oE + mono4_index<D>(pair_a<D>(p), pair_b<D>(p), pair_a<D>(q), pair_b<D>(q))) * n + i];

    // Q^T = L B (d x m);  M = E - C Q^T;  CL = C L (m x d)
    double Qt[d][m], CL[m][d];
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
        for (int p = 0; p < m; ++p) {
            double t = 0.0;
#pragma unroll
            for (int b = 0; b < d; ++b) t += sym_at<D>(L, a, b) * Bt[b][p];
            Qt[a][p] = t;
        }
#pragma unroll
    for (int p = 0; p < m; ++p) {
#pragma unroll
        for (int q = 0; q < m; ++q) {
            double t = 0.0;
#pragma unroll
            for (int a = 0; a < d; ++a) t += Ct[p][a] * Qt[a][q];
            M[p][q] -= t;
        }
#pragma unroll
        for (int a = 0; a < d; ++a) {
            double t = 0.0;
#pragma unroll
            for (int b = 0; b < d; ++b) t += Ct[p][b] * sym_at<D>(L, b, a);
            CL[p][a] = t;
        }
    }
    // Q^T and C L wait in LDS (one column per thread) while M is inverted and
    // are read back per output column, which keeps them out of registers
    __shared__ double sQC[2 * d * m][128];
    const int tq = threadIdx.x;
#pragma unroll
    for (int a = 0; a < d; ++a)
#pragma unroll
        for (int p = 0; p < m; ++p) {
            sQC[a * m + p][tq] = Qt[a][p];
            sQC[d * m + p * d + a][tq] = CL[p][a];
        }
    asm volatile("" ::: "memory");
    if (!fl && !gj_invert<m>(M)) fl |= VCT_FLAG_SINGULAR_M;   // M now holds M^-1
    asm volatile("" ::: "memory");

    // VCT coefficients at the particle
    const double x = pos[i], y = (D == 3) ? pos[n + i] : 0.0, zh = pos[(int64_t)(D - 1) * n + i];
    const MapCoef<double> mc = map_coef_at(mp, i, x, y, zh);
    // Sec. 2.1 requires alpha > 0 (a dry sigma column without the limiter
    // gives alpha <= 0 or infinite); such a particle is flagged
    if (!(mc.alpha > 0.0) || !isfinite(mc.alpha + mc.gx + mc.gy + mc.c0 + mc.zxy)) fl |= VCT_FLAG_MAP;
    const bool grad1 = (o1.mask & VCT_OPT_GRAD1) != 0;
    const double invR2 = invR * invR;
    const double nanv = __builtin_nan("");
    // one state's rows of output group k (or of W when w is set)
    auto put = [&](const SolveOut& so, int k, bool w, const double* pg, const double* ph) {
        const int base = w ? nL + so.nrows * nk : nL;
        const int stride = w ? d : nk;
        emit_rows<D>(so.mask, mc, pg, ph, [&](int o, double v) {
            v = fl ? nanv : v;
            const int64_t idx = (int64_t)(base + o * stride + k) * n + i;
            if (so.s64) so.s64[idx] = v;
            if (so.s32) so.s32[idx] = (float)v;
        });
    };

#pragma unroll
    for (int k = 0; k < nk; ++k) {
        // z = M^-1 (C L e_k) for the first-order sums, the column of M^-1 for the others
        double z[m];
        if (k < d) {
            double cl[m];
#pragma unroll
            for (int q = 0; q < m; ++q) cl[q] = sQC[d * m + q * d + k][tq];
#pragma unroll
            for (int p = 0; p < m; ++p) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < m; ++q) t += M[p][q] * cl[q];
                z[p] = t;
            }
        } else {
#pragma unroll
            for (int p = 0; p < m; ++p) z[p] = M[p][k - d];
        }
        double pg[d], ph[m];
#pragma unroll
        for (int a = 0; a < d; ++a) {
            double t = 0.0;
#pragma unroll
            for (int p = 0; p < m; ++p) t += sQC[a * m + p][tq] * z[p];
            double g;
            if (k < d) g = sym_at<D>(L, a, k) + (grad1 ? 0.0 : t);
            else g = grad1 ? 0.0 : -t;
            pg[a] = g * invR;
        }
#pragma unroll
        for (int p = 0; p < m; ++p) {
            const double hv = (k < d) ? -z[p] : z[p];
            ph[p] = hv * ((p < d) ? 2.0 * invR2 : invR2);
        }
        put(o1, k, false, pg, ph);
        if constexpr (TWO) put(o2, k, false, pg, ph);
    }
    // W: response of every output row to a unit projected gradient (a linear
    // field), used by the apply kernels to add back the linear part removed
    // from the field before the neighbour sums
#pragma unroll
    for (int a = 0; a < d; ++a) {
        double pg[d], ph[m];
#pragma unroll
        for (int b = 0; b < d; ++b) pg[b] = (a == b) ? 1.0 : 0.0;
#pragma unroll
        for (int p = 0; p < m; ++p) ph[p] = 0.0;
        put(o1, a, true, pg, ph);
        if constexpr (TWO) put(o2, a, true, pg, ph);
    }
#pragma unroll
    for (int p = 0; p < nL; ++p) {
        const double v = fl ? nanv : L[p];
        if (o1.s64) o1.s64[(int64_t)p * n + i] = v;
        if (o1.s32) o1.s32[(int64_t)p * n + i] = (float)v;
        if constexpr (TWO) {
            if (o2.s64) o2.s64[(int64_t)p * n + i] = v;
            if (o2.s32) o2.s32[(int64_t)p * n + i] = (float)v;
        }
    }
    if (flags_out) flags_out[i] = (uint8_t)fl;
    if (fl && nflag) atomicAdd(nflag, 1ull);
}

int nlist_check(const vct_nlist* nl, Grid& g);

template <int D>
static int launch_solve(int64_t n, const double* pos, const double* mom, const uint8_t* mflags, double invR,
                        const MapParams& mp, const SolveOut& o1, const SolveOut& o2, uint8_t* flags,
                        unsigned long long* nflag, hipStream_t s) {
    const int64_t nb2 = (n + 127) / 128;
    if (o2.s64 || o2.s32)
        VCT_LAUNCH("k_moment_solve (two states)", (k_moment_solve<D, true>), dim3((unsigned)nb2), dim3(128), 0, s,
                   n, pos, mom, mflags, invR, mp, o1, o2, flags, nflag);
    else
        VCT_LAUNCH("k_moment_solve", (k_moment_solve<D, false>), dim3((unsigned)nb2), dim3(128), 0, s, n, pos,
                   mom, mflags, invR, mp, o1, o2, flags, nflag);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

template <int D, int KERNEL>
static int launch_moments(const vct_nlist* nl, const Grid& g, const double* pos, const double* vol, double invR,
                          const MapParams& mp, const SolveOut& o1, const SolveOut& o2, double* mom, uint8_t* mflags,
                          uint8_t* flags, unsigned long long* nflag, hipStream_t s) {
    const int64_t n = nl->n;
    const int64_t ncols = D == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    SweepArgs a;
    a.n = n; a.invR = invR; a.g = g; a.pos = pos; a.vol = vol; a.row_ptr = nl->row_ptr; a.col16 = nl->col16;
    a.cs = nl->cell_start; a.cstart = nl->chunk_start; a.cinfo = reinterpret_cast<const int4*>(nl->chunk_info);
    a.cwin = nl->chunk_win;
    a.nchunks = nl->chunk_off + ncols; a.mom = mom; a.mflags = mflags;
    const int64_t cap = ncols + n / kChunk + 1;
    VCT_LAUNCH("k_moment_sweeps", (k_moment_sweeps<D, KERNEL>), dim3((unsigned)cap), dim3(kMThreads), 0, s, a);
    VCT_LAUNCH_CHECK();
    return launch_solve<D>(n, pos, mom, mflags, invR, mp, o1, o2, flags, nflag, s);
}

VCT_CHECKS_TU(checks_moments)

}  // namespace vct

using namespace vct;

extern "C" size_t vct_moments_workspace_size(int dim, int64_t n) {
    if ((dim != 2 && dim != 3) || n < 0) return 0;
    int total = dim == 2 ? MomLayout<2>::total : MomLayout<3>::total;
    return aligned_sum({(size_t)n * total * sizeof(double), (size_t)n, 64});
}

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

static int moments_impl(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                        const vct_map* map, uint32_t out_mask, double* state64, float* state32, uint32_t out_mask2,
                        double* state64_2, float* state32_2, uint8_t* flags, int64_t* n_flagged, void* ws,
                        size_t ws_bytes, void* stream) {
    Grid g;
    int st = nlist_check(nl, g);
    if (st) return st;
    const int dim = nl->dim;
    const int64_t n = nl->n;
    if (!map || !mask_valid(out_mask) || (kernel != VCT_KERNEL_WENDLAND_C2 && kernel != VCT_KERNEL_CUBIC_SPLINE))
        return VCT_E_ARG;
    const bool two = state64_2 || state32_2;
    if (two && (!mask_valid(out_mask2) || ((out_mask ^ out_mask2) & VCT_OPT_GRAD1))) return VCT_E_ARG;
    MapParams mp;
    st = map_params_from(map, dim, n, mp);
    if (st) return st;
    if (n > 0 && (!pos_sorted || !vol_sorted || !nl->col16 || (!state64 && !state32))) return VCT_E_ARG;
    if (!ws || ws_bytes < vct_moments_workspace_size(dim, n)) return VCT_E_WORKSPACE;
    hipStream_t s = as_stream(stream);
    Carver cv(ws, ws_bytes);
    const int total = dim == 2 ? MomLayout<2>::total : MomLayout<3>::total;
    double* mom = cv.take<double>((size_t)n * total);
    uint8_t* mflags = cv.take<uint8_t>((size_t)n);
    unsigned long long* cnt = cv.take<unsigned long long>(8);
    VCT_LAUNCH("k_zero_u64", k_zero_u64, dim3(1), dim3(1), 0, s, cnt);
    VCT_LAUNCH_CHECK();
    if (n > 0) {
        const double invR = 1.0 / nl->R;
        const SolveOut o1{out_mask, n_out_rows(dim, out_mask), state64, state32};
        const SolveOut o2{two ? out_mask2 : 0u, two ? n_out_rows(dim, out_mask2) : 0, state64_2, state32_2};
        if (dim == 2)
            st = (kernel == VCT_KERNEL_WENDLAND_C2)
                     ? launch_moments<2, VCT_KERNEL_WENDLAND_C2>(nl, g, pos_sorted, vol_sorted, invR, mp, o1, o2, mom,
                                                                 mflags, flags, cnt, s)
                     : launch_moments<2, VCT_KERNEL_CUBIC_SPLINE>(nl, g, pos_sorted, vol_sorted, invR, mp, o1, o2,
                                                                  mom, mflags, flags, cnt, s);
        else
            st = (kernel == VCT_KERNEL_WENDLAND_C2)
                     ? launch_moments<3, VCT_KERNEL_WENDLAND_C2>(nl, g, pos_sorted, vol_sorted, invR, mp, o1, o2, mom,
                                                                 mflags, flags, cnt, s)
                     : launch_moments<3, VCT_KERNEL_CUBIC_SPLINE>(nl, g, pos_sorted, vol_sorted, invR, mp, o1, o2,
                                                                  mom, mflags, flags, cnt, s);
        if (st) return st;
    }
    if (n_flagged) {
        unsigned long long h = 0;
        VCT_HIP_CHECK(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
        VCT_HIP_CHECK(hipStreamSynchronize(s));
        *n_flagged = (int64_t)h;
        return h ? VCT_W_FLAGGED : VCT_OK;
    }
    return VCT_OK;
}

extern "C" int vct_moments(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                           const vct_map* map, uint32_t out_mask, double* state64, float* state32, uint8_t* flags,
                           int64_t* n_flagged, void* ws, size_t ws_bytes, void* stream) {
    VCT_API_RANGE("vct_moments");
    return moments_impl(nl, pos_sorted, vol_sorted, kernel, map, out_mask, state64, state32, 0u, nullptr, nullptr,
                        flags, n_flagged, ws, ws_bytes, stream);
}

extern "C" int vct_moments_ex(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                              const vct_map* map, uint32_t out_mask, double* state64, float* state32,
                              uint32_t out_mask2, double* state64_2, float* state32_2, uint8_t* flags,
                              int64_t* n_flagged, void* ws, size_t ws_bytes, void* stream) {
    VCT_API_RANGE("vct_moments_ex");
    return moments_impl(nl, pos_sorted, vol_sorted, kernel, map, out_mask, state64, state32, out_mask2, state64_2,
                        state32_2, flags, n_flagged, ws, ws_bytes, stream);
}

extern "C" int vct_moments_resolve(const vct_nlist* nl, const double* pos_sorted, const vct_map* map,
                                   uint32_t out_mask, double* state64, float* state32, uint8_t* flags,
                                   int64_t* n_flagged, void* ws, size_t ws_bytes, void* stream) {
    VCT_API_RANGE("vct_moments_resolve");
    Grid g;
    int st = nlist_check(nl, g);
    if (st) return st;
    const int dim = nl->dim;
    const int64_t n = nl->n;
    if (!map || !mask_valid(out_mask)) return VCT_E_ARG;
    MapParams mp;
    st = map_params_from(map, dim, n, mp);
    if (st) return st;
    if (n > 0 && (!pos_sorted || (!state64 && !state32))) return VCT_E_ARG;
    if (!ws || ws_bytes < vct_moments_workspace_size(dim, n)) return VCT_E_WORKSPACE;
    hipStream_t s = as_stream(stream);
    // the same carving as vct_moments: the sums and sweep flags it left behind
    Carver cv(ws, ws_bytes);
    const int total = dim == 2 ? MomLayout<2>::total : MomLayout<3>::total;
    const double* mom = cv.take<double>((size_t)n * total);
    const uint8_t* mflags = cv.take<uint8_t>((size_t)n);
    unsigned long long* cnt = cv.take<unsigned long long>(8);
    VCT_LAUNCH("k_zero_u64", k_zero_u64, dim3(1), dim3(1), 0, s, cnt);
    VCT_LAUNCH_CHECK();
    if (n > 0) {
        const double invR = 1.0 / nl->R;
        const SolveOut o1{out_mask, n_out_rows(dim, out_mask), state64, state32};
        const SolveOut o2{0u, 0, nullptr, nullptr};
        st = dim == 2 ? launch_solve<2>(n, pos_sorted, mom, mflags, invR, mp, o1, o2, flags, cnt, s)
                      : launch_solve<3>(n, pos_sorted, mom, mflags, invR, mp, o1, o2, flags, cnt, s);
        if (st) return st;
    }
    if (n_flagged) {
        unsigned long long h = 0;
        VCT_HIP_CHECK(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
        VCT_HIP_CHECK(hipStreamSynchronize(s));
        *n_flagged = (int64_t)h;
        return h ? VCT_W_FLAGGED : VCT_OK;
    }
    return VCT_OK;
}
