// Operator application (paper Sec. 3.1, Eqs. gra_1st and sec_SPH2; Sec. 2.1,
// Eqs. grad_VCT and lap_VCT): the neighbour sums [a_i; s_i] of each field,
// then out_i = P_i [a_i; s_i] with the per-particle state of vct_moments.
//
// Numerics.  phi_ij is dominated by its first-order part r_ij . grad phi,
// which cancels across a (nearly) symmetric neighbourhood in s_i; rounding the
// individual terms is then amplified by |grad phi| / (R |Hess phi|).  The
// operator is linear and reproduces linear fields exactly, so for any vector
// G, out(phi) = P [a; s](psi) + W G with psi_ij = phi_ij - (x_j - x_i) . G and
// W the response of the output rows to a unit projected gradient (stored by
// vct_moments).  The kernel sums in two passes: pass 1 forms the particle's
// first-order gradient G = L a (d sums), pass 2 sums the residual psi, which
// is second-order small and has a(psi) = 0 up to rounding.  psi is formed in
// FP64 from the FP64 positions and field values; the pair geometry, kernel and
// sums run in the arithmetic type T (FP64, or FP32 for the mixed form).  The
// result is the same linear operator; only the rounding changes.
//
// Work decomposition.  One work-group per chunk (at most 64 consecutive
// particles of one cell column).  The chunk's neighbour window (positions,
// field values, volumes) and its block of 16-bit row entries are staged once
// in LDS with coalesced loads; each particle is served by kLanes lanes that
// hold their share of the row entries in registers and read the pair records
// from LDS, software-pipelined one record ahead.  The group reduces its sums
// with cross-lane shuffles; the products with the state are done with one
// thread per (row, particle) so that the state is read with unit stride.
// Work-groups are remapped so each XCD covers a contiguous range of chunks.
#include <type_traits>

#include "common.h"
#include "tiles.h"

namespace vct {

int nlist_check(const vct_nlist* nl, Grid& g);

constexpr int kColCap = 7168;                // row entries of a chunk staged in LDS

// Lanes per particle, register slots per lane, occupancy target (waves per
// SIMD) and LDS window capacity (records) of each arithmetic type
// (overridable at build time for tuning).  Both forms run 512-thread groups
// (8 lanes per particle) at 4 waves per SIMD, two groups per CU.  The FP64
// form's FP64 records and sums take a smaller window (about 77 KB of LDS per
// group) and fill the 128 VGPRs that 4 waves allow (a few prologue and
// epilogue values go to scratch, none of the pair loops' values).
#ifndef VCT_APPLY_F_LANES
#define VCT_APPLY_F_LANES 8
#endif
#ifndef VCT_APPLY_F_SLOTS
#define VCT_APPLY_F_SLOTS 14
#endif
#ifndef VCT_APPLY_F_WAVES
#define VCT_APPLY_F_WAVES 4
#endif
#ifndef VCT_APPLY_F_WIN
#define VCT_APPLY_F_WIN 1664
#endif
#ifndef VCT_APPLY_D_LANES
#define VCT_APPLY_D_LANES 8
#endif
#ifndef VCT_APPLY_D_SLOTS
#define VCT_APPLY_D_SLOTS 14
#endif
#ifndef VCT_APPLY_D_WAVES
#define VCT_APPLY_D_WAVES 4
#endif
#ifndef VCT_APPLY_D_WIN
#define VCT_APPLY_D_WIN 1400
#endif
#ifndef VCT_APPLY_F_COLS
#define VCT_APPLY_F_COLS true
#endif
#ifndef VCT_APPLY_D_COLS
#define VCT_APPLY_D_COLS true
#endif
template <class T> struct ApplyCfg;
template <> struct ApplyCfg<float> {
    static constexpr int lanes = VCT_APPLY_F_LANES;
    static constexpr int slots = VCT_APPLY_F_SLOTS;
    static constexpr int waves = VCT_APPLY_F_WAVES;
    static constexpr int win = VCT_APPLY_F_WIN;
    static constexpr bool col_lds = VCT_APPLY_F_COLS;   // stage the chunk's row entries in LDS
    static constexpr int threads = kChunk * lanes;   // one chunk per work-group
};
template <> struct ApplyCfg<double> {
    static constexpr int lanes = VCT_APPLY_D_LANES;
    static constexpr int slots = VCT_APPLY_D_SLOTS;
    static constexpr int waves = VCT_APPLY_D_WAVES;
    static constexpr int win = VCT_APPLY_D_WIN;
    static constexpr bool col_lds = VCT_APPLY_D_COLS;
    static constexpr int threads = kChunk * lanes;
};

template <class S> struct ApplyArgs {
    int64_t n;
    int nf;
    int nrows;
    double invR;
    Grid g;
    const double* phi;
    const double* pos;
    const double* vol;
    const int64_t* row_ptr;
    const uint16_t* col16;
    const int64_t* cs;
    const int32_t* cstart;
    const int4* cinfo;
    const int32_t* cwin;   // stored windows or NULL
    const int64_t* nchunks;
    const S* state;
    double* out;
    float* g_out;        // [nf][D][n] or NULL: the first pass's G~, written
    const float* g_in;   // [nf][D][n] or NULL: G~ given to the FP64 form (first pass skipped)
};

// The mixed form keeps positions in units of R (x / R, in FP64): the FP64
// offset is then r~ itself and only needs rounding to FP32.  The FP64 form
// keeps positions as they are, so its offsets are exact differences.
template <class T> struct Scaled {
    static constexpr bool value = std::is_same<T, float>::value;
};

// Pair geometry: FP64 offset dx = x_j - x_i (in units of R for the mixed
// form), r~ = dx / R, q^2 = |r~|^2 and V_j c~(q) in the arithmetic type T;
// with IQ4 also 1 / q^4, both from one reciprocal square root.  An empty
// register slot (use false) takes q^2 = 4, outside the support: c~ = 0
// exactly, 1 / q^4 stays finite, and its terms add zero without a mask on
// each product.
template <int D, int KERNEL, class T, bool IQ4 = false>
__device__ __forceinline__ void pair_geom(const double4& q, T vj, const double (&xi)[3], T invR,
                                          double (&dx)[D], T (&r)[D], T& q2, T& vc, T* iq4 = nullptr,
                                          bool use = true) {
    dx[0] = q.x - xi[0];
    dx[1] = q.y - xi[1];
    if (D == 3) dx[D - 1] = q.z - xi[2];
    q2 = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        r[a] = Scaled<T>::value ? T(dx[a]) : T(dx[a]) * invR;
        q2 += r[a] * r[a];
    }
    q2 = use ? q2 : T(4);
    if (IQ4) {
        T rs;
        if constexpr (Scaled<T>::value) rs = __builtin_amdgcn_rsqf(q2);
        else rs = vrsq(q2);
        const T rs2 = rs * rs;
        vc = vj * kernel_shape<KERNEL>(q2 * rs);
        *iq4 = rs2 * rs2;
    } else {
        vc = vj * kernel_shape<KERNEL>(vsqrt(q2));
    }
}

// Sums of one pair with residual psi: a~ += V c~ psi r~ and
// s~ += V c~ psi (r~' L~ r~) / |r~|^4 r~ r~' (L2 holds L~ with doubled
// off-diagonal entries), with vq = V c~ / |r~|^4 given.
template <int D, class T>
__device__ __forceinline__ void pair_sums(const T (&r)[D], T vq, T vc, T psi, const T (&L2)[Dims<D>::nL],
                                          T (&acc)[Dims<D>::nk]) {
    using Dm = Dims<D>;
    T qv[Dm::m];
#pragma unroll
    for (int p = 0; p < Dm::m; ++p) qv[p] = r[pair_a<D>(p)] * r[pair_b<D>(p)];
    T rLr = T(0);
#pragma unroll
    for (int p = 0; p < Dm::nL; ++p) rLr += L2[p] * qv[p];
    const T wa = vc * psi, ws = vq * psi * rLr;
#pragma unroll
    for (int a = 0; a < D; ++a) acc[a] += wa * r[a];
#pragma unroll
    for (int p = 0; p < Dm::m; ++p) acc[D + p] += ws * qv[p];
}

// G~ = L~ a~ after the group reduction of a~ (dimensionless).
template <int D, class T>
__device__ __forceinline__ void group_gradient(const T (&L2)[Dims<D>::nL], T (&a1)[D], T (&Gt)[D]) {
#pragma unroll
    for (int a = 0; a < D; ++a) a1[a] = group_sum(a1[a], ApplyCfg<T>::lanes);
#pragma unroll
    for (int a = 0; a < D; ++a) {
        T t = T(0);
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const int p = sym_index<D>(a, c);
            t += (a == c ? L2[p] : T(0.5) * L2[p]) * a1[c];
        }
        Gt[a] = t;
    }
}

template <int D, class T, class S>
__device__ __forceinline__ void load_L(const ApplyArgs<S>& A, int64_t ii, T (&L2)[Dims<D>::nL]) {
#pragma unroll
    for (int p = 0; p < Dims<D>::nL; ++p) {
        const T v = T(A.state[(int64_t)p * A.n + ii]);
        L2[p] = (pair_a<D>(p) == pair_b<D>(p)) ? v : T(2) * v;
    }
}

// out row o of particle i: P_o [a~; s~] + W_o G~ / R.
template <int D, class T, class S>
__device__ __forceinline__ double out_row(const ApplyArgs<S>& A, int64_t i, int o, const T* acc, const T* Gt) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, nk = Dm::nk;
    const int64_t n = A.n;
    const S* P = A.state + (int64_t)(nL + o * nk) * n + i;
    const S* Wr = A.state + (int64_t)(nL + A.nrows * nk + o * D) * n + i;
    T v = T(0);
#pragma unroll
    for (int c = 0; c < nk; ++c) v += T(P[(int64_t)c * n]) * acc[c];
    T lin = T(0);
#pragma unroll
    for (int a = 0; a < D; ++a) lin += T(Wr[(int64_t)a * n]) * Gt[a];
    return (double)v + (double)lin * A.invR;
}

// What a launch does with the first-pass gradient G~: nothing, read it
// (FP64 form: the first pass is skipped) or write it.  Separate
// instantiations, so that a form without the gradient pays no registers for it.
enum { kGNone = 0, kGIn = 1, kGOut = 2 };

// A chunk whose window exceeds the LDS capacity: the same two passes with
// every record read from the memory hierarchy.
template <int D, int KERNEL, class T, class S, bool GOUT>
__device__ __forceinline__ void apply_chunk_global(const ApplyArgs<S>& A, const WindowT<D>& w, int64_t p0,
                                                int64_t p1) {
    constexpr int nk = Dims<D>::nk, kLanes = ApplyCfg<T>::lanes;
    const int64_t n = A.n;
    const int lane = threadIdx.x % kLanes;
    const int64_t i = p0 + threadIdx.x / kLanes;
    if (i >= p1) return;   // whole groups leave together
    const T invR = T(A.invR);
    const double ps = Scaled<T>::value ? A.invR : 1.0;   // position scale
    double xi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xi[a] = a < D ? A.pos[a * n + i] * ps : 0.0;
    T L2[Dims<D>::nL];
    load_L<D, T, S>(A, i, L2);
    const int64_t rb = A.row_ptr[i], re = A.row_ptr[i + 1];
    for (int f = 0; f < A.nf; ++f) {
        const double* ph = A.phi + (int64_t)f * n;
        const double phi_i = ph[i];
        auto fetch = [&](int t, double4& q, T& v) {
            const int64_t j = window_global<D>(w, t);
            q = make_double4(A.pos[j] * ps, A.pos[n + j] * ps, D == 3 ? A.pos[2 * n + j] * ps : 0.0, ph[j]);
            v = T(A.vol[j]);
        };
        T a1[D], Gt[D];
#pragma unroll
        for (int a = 0; a < D; ++a) a1[a] = T(0);
        for (int64_t e = rb + lane; e < re; e += kLanes) {
            double4 q;
            T vj, r[D], q2, vc;
            double dx[D];
            fetch(A.col16[e], q, vj);
            pair_geom<D, KERNEL, T>(q, vj, xi, invR, dx, r, q2, vc);
            const T wgt = vc * T(q.w - phi_i);
#pragma unroll
            for (int a = 0; a < D; ++a) a1[a] += wgt * r[a];
        }
        group_gradient<D, T>(L2, a1, Gt);
        if (GOUT && lane == 0) {
#pragma unroll
            for (int a = 0; a < D; ++a) A.g_out[((int64_t)f * D + a) * n + i] = (float)Gt[a];
        }
        double Gp[D];
#pragma unroll
        for (int a = 0; a < D; ++a) Gp[a] = Scaled<T>::value ? (double)Gt[a] : (double)Gt[a] * A.invR;
        T acc[nk];
#pragma unroll
        for (int c = 0; c < nk; ++c) acc[c] = T(0);
        for (int64_t e = rb + lane; e < re; e += kLanes) {
            double4 q;
            T vj, r[D], q2, vc;
            double dx[D];
            fetch(A.col16[e], q, vj);
            T iq4;
            pair_geom<D, KERNEL, T, true>(q, vj, xi, invR, dx, r, q2, vc, &iq4);
            double psi = q.w - phi_i;
#pragma unroll
            for (int a = 0; a < D; ++a) psi -= dx[a] * Gp[a];
            pair_sums<D, T>(r, vc * iq4, vc, T(psi), L2, acc);
        }
#pragma unroll
        for (int c = 0; c < nk; ++c) acc[c] = group_sum(acc[c], kLanes);
        for (int o = lane; o < A.nrows; o += kLanes)
            A.out[((int64_t)f * n + i) * A.nrows + o] = out_row<D, T, S>(A, i, o, acc, Gt);
    }
}

// GM (kGNone, kGIn, kGOut): what the launch does with G~.
template <int D, int KERNEL, class T, class S, int GM>
__global__ __launch_bounds__(ApplyCfg<T>::threads, ApplyCfg<T>::waves) void k_apply(ApplyArgs<S> A) {
    constexpr bool GIN = GM == kGIn, GOUT = GM == kGOut;
    static_assert(!GIN || !Scaled<T>::value, "only the FP64 form takes a given gradient");
    using Dm = Dims<D>;
    constexpr int nk = Dm::nk, kS = ApplyCfg<T>::slots, kW = ApplyCfg<T>::win;
    constexpr int kLanes = ApplyCfg<T>::lanes, kThreads = ApplyCfg<T>::threads;
    constexpr int kColBlocks = (kColCap / 8 + kThreads - 1) / kThreads;   // 16-byte blocks per thread
    __shared__ double4 sd[kW];
    __shared__ T sv[kW];
    __shared__ uint4 scol4[ApplyCfg<T>::col_lds ? kColCap / 8 : 1];
    __shared__ T sacc[kChunk][nk + D];
    __shared__ WindowT<D> w;
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *A.nchunks) return;   // uniform over the work-group
    const int64_t n = A.n;
    const int64_t p0 = A.cstart[b], p1 = A.cstart[b + 1];
    if (threadIdx.x < kWave) {
        if (A.cwin) window_load<D>(A.cwin, b, w);
        else chunk_window_wave<D>(A.g, A.cs, A.cinfo[b], w);
    }
    // per-particle data, requested while the window is formed
    const int lane = threadIdx.x % kLanes;
    const int pl = threadIdx.x / kLanes;
    const int64_t i = p0 + pl;
    const bool valid = i < p1;
    const int64_t ii = valid ? i : p0;
    const double ps = Scaled<T>::value ? A.invR : 1.0;   // position scale
    double xi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xi[a] = a < D ? A.pos[a * n + ii] * ps : 0.0;
    T L2[Dm::nL];
    load_L<D, T, S>(A, ii, L2);
    const int64_t rb = valid ? A.row_ptr[ii] : 0, re = valid ? A.row_ptr[ii + 1] : 0;
    // the chunk's row entries [cb, ce), staged from the 16-byte aligned cb8
    const int64_t cb = A.row_ptr[p0], ce = A.row_ptr[p1], nnz = A.row_ptr[n];
    const int64_t cb8 = cb & ~int64_t(7);
    const bool col_lds = ApplyCfg<T>::col_lds && ce - cb8 <= kColCap;
    __syncthreads();
    const int W = __builtin_amdgcn_readfirstlane(w.off[w.nr]);
    if (W > kW) {
        apply_chunk_global<D, KERNEL, T, S, GOUT>(A, w, p0, p1);
        return;
    }
    // stage the window records and the chunk's row entries, in batches of
    // loads that are all issued before the batch's first LDS store
    {
        constexpr int kRep = (kW + kThreads - 1) / kThreads;
        constexpr int kBatch = kRep < 4 ? kRep : 4;
        const double* ph = A.phi;
        uint4 cv[kColBlocks];
        if (col_lds) {
#pragma unroll
            for (int k = 0; k < kColBlocks; ++k) {
                const int blk = threadIdx.x + k * kThreads;
                const int64_t base = cb8 + 8 * (int64_t)blk;
                if (base < ce) {
                    if (base + 8 <= nnz) {
                        cv[k] = *reinterpret_cast<const uint4*>(A.col16 + base);
                    } else {   // the last block of the array: entry by entry
                        uint32_t h[4] = {0u, 0u, 0u, 0u};
                        for (int u = 0; u < 8 && base + u < nnz; ++u)
                            h[u / 2] |= (uint32_t)A.col16[base + u] << (16 * (u % 2));
                        cv[k] = make_uint4(h[0], h[1], h[2], h[3]);
                    }
                }
            }
        }
#pragma unroll
        for (int k0 = 0; k0 < kRep; k0 += kBatch) {
            double4 q[kBatch];
            T v[kBatch];
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int t = threadIdx.x + (k0 + k) * kThreads;
                if (t < W) {   // lanes past the window load nothing (whole waves skip)
                    const int64_t j = window_global<D>(w, t);
                    q[k] = make_double4(A.pos[j] * ps, A.pos[n + j] * ps, D == 3 ? A.pos[2 * n + j] * ps : 0.0,
                                        ph[j]);
                    v[k] = T(A.vol[j]);
                }
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int t = threadIdx.x + (k0 + k) * kThreads;
                if (t < W) {
                    sd[t] = q[k];
                    sv[t] = v[k];
                }
            }
        }
        if (col_lds) {
#pragma unroll
            for (int k = 0; k < kColBlocks; ++k) {
                const int blk = threadIdx.x + k * kThreads;
                if (cb8 + 8 * (int64_t)blk < ce) scol4[blk] = cv[k];
            }
        }
    }
    __syncthreads();
    // register slots: entry rb + lane + kLanes s; an empty slot repeats the
    // row's first entry (offset 0 for an empty row) and is masked out
    const uint16_t* scol = reinterpret_cast<const uint16_t*>(scol4);
    auto col_at = [&](int64_t e) -> int {
        return dcheck(col_lds ? (int)scol[e - cb8] : (int)A.col16[e], W, kChkWindow);
    };
    // (two 16-bit offsets per register)
    uint32_t cpk[(kS + 1) / 2];
    int nslot = 0;
    {
        const uint32_t first = re > rb ? (uint32_t)col_at(rb) : 0u;
        const int len = (int)(re - rb);   // 32-bit row-local indices: one LDS base, immediate offsets
        const uint16_t* srow = scol + (col_lds ? (int)(rb - cb8) : 0) + lane;
#pragma unroll
        for (int s = 0; s < kS; ++s) {
            const int idx = lane + kLanes * s;
            const bool in = idx < len;
            const uint32_t c = in ? (col_lds ? (uint32_t)srow[kLanes * s] : (uint32_t)A.col16[rb + idx]) : first;
            nslot += in ? 1 : 0;
            if (s % 2 == 0) cpk[s / 2] = c;
            else cpk[s / 2] |= c << 16;
        }
    }
    auto cols = [&](int s) -> int { return dcheck((int)((cpk[s / 2] >> (16 * (s % 2))) & 0xffffu), W, kChkWindow); };
    const int64_t tail = rb + (int64_t)kLanes * kS;
    const T invR = T(A.invR);
    for (int f = 0; f < A.nf; ++f) {
        const double* ph = A.phi + (int64_t)f * n;
        if (f > 0) {
            // every read of sd happened before the epilogue's barrier
            for (int t = threadIdx.x; t < W; t += kThreads) sd[t].w = ph[window_global<D>(w, t)];
            __syncthreads();
        }
        const double phi_i = ph[ii];
        // pass 1: first-order sums and G~ = L~ a~, in FP32 for both forms.  G
        // only sets the residual psi of pass 2; out = P [a; s](psi) + W G
        // holds for any G, so an FP32 G leaves the FP64 form's sums FP64 and
        // its result as accurate (psi keeps a linear part of relative size
        // 1e-7, which the operator reproduces exactly).
        float a1[D];
        T Gt[D];
#pragma unroll
        for (int a = 0; a < D; ++a) a1[a] = 0.0f;
        const float invRf = (float)A.invR;
        // The mixed form keeps each register slot's V_j c~ and V_j c~ / q^4
        // from pass 1, so pass 2 forms neither (the FP64 form needs its own
        // FP64 values).
        float vcs[kS], vqs[kS];
        auto term1 = [&](const double4& q, T vj, bool use, float& vq) -> float {
            if constexpr (Scaled<T>::value) {
                double dx[D];
                T r[D], q2, vc, iq4;
                pair_geom<D, KERNEL, T, true>(q, vj, xi, invR, dx, r, q2, vc, &iq4, use);
                vq = vc * iq4;
                const T wgt = vc * T(q.w - phi_i);
#pragma unroll
                for (int a = 0; a < D; ++a) a1[a] += wgt * r[a];
                return vc;
            } else {
                float r[D], q2 = 0.0f;
                r[0] = (float)(q.x - xi[0]) * invRf;
                r[1] = (float)(q.y - xi[1]) * invRf;
                if (D == 3) r[D - 1] = (float)(q.z - xi[2]) * invRf;
#pragma unroll
                for (int a = 0; a < D; ++a) q2 += r[a] * r[a];
                q2 = use ? q2 : 4.0f;
                const float vc = (float)vj * kernel_shape<KERNEL>(vsqrt(q2));
                const float wgt = vc * (float)(q.w - phi_i);
#pragma unroll
                for (int a = 0; a < D; ++a) a1[a] += wgt * r[a];
                vq = 0.0f;
                return 0.0f;
            }
        };
        // The FP64 form given G~ (a mixed call's first pass on the same field
        // and geometry) skips its own: any G gives the same result up to the
        // rounding of psi.
        if constexpr (GIN) {
#pragma unroll
            for (int a = 0; a < D; ++a) Gt[a] = T(A.g_in[((int64_t)f * D + a) * n + ii]);
        } else {
            // software pipeline: the record of slot s + 1 is read while slot s
            // is summed (the scheduling barriers keep the compiler from
            // hoisting every slot's read, which would exhaust the registers)
            double4 qn = sd[cols(0)];
            T vn = sv[cols(0)];
#pragma unroll
            for (int s = 0; s < kS; ++s) {
                const double4 q = qn;
                const T vj = vn;
                if (s + 1 < kS) {
                    qn = sd[cols(s + 1)];
                    vn = sv[cols(s + 1)];
                }
                __builtin_amdgcn_sched_barrier(0);
                vcs[s] = term1(q, vj, s < nslot, vqs[s]);
                __builtin_amdgcn_sched_barrier(0);
            }
            for (int64_t e = tail + lane; e < re; e += kLanes) {
                const int t = col_at(e);
                float vq_;
                term1(sd[t], sv[t], true, vq_);
            }
#pragma unroll
            for (int a = 0; a < D; ++a) a1[a] = group_sum(a1[a], kLanes);
#pragma unroll
            for (int a = 0; a < D; ++a) {
                T t = T(0);
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    const int p = sym_index<D>(a, c);
                    t += (a == c ? L2[p] : T(0.5) * L2[p]) * T(a1[c]);
                }
                Gt[a] = t;
            }
        }
        double Gp[D];
#pragma unroll
        for (int a = 0; a < D; ++a) Gp[a] = Scaled<T>::value ? (double)Gt[a] : (double)Gt[a] * A.invR;
        // G~ waits for the epilogue in LDS, not in registers
        if (lane == 0) {
#pragma unroll
            for (int a = 0; a < D; ++a) sacc[pl][nk + a] = Gt[a];
        }
        // pass 2: sums of the residual psi_ij = phi_ij - (x_j - x_i) . G.
        // The empty asm makes the packed offsets opaque, so the record
        // addresses are recomputed here instead of being kept live from pass 1.
#pragma unroll
        for (int k = 0; k < (kS + 1) / 2; ++k) asm volatile("" : "+v"(cpk[k]));
        T acc[nk];
#pragma unroll
        for (int c = 0; c < nk; ++c) acc[c] = T(0);
        auto term2 = [&](const double4& q, T vj, bool use, int s) {
            double dx[D];
            T r[D], q2, vc;
            T iq4;
            if (Scaled<T>::value && s >= 0) {   // V c~ and V c~ / q^4 from pass 1
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    dx[a] = (a == 0 ? q.x : a == 1 ? q.y : q.z) - xi[a];
                    r[a] = T(dx[a]);
                }
                vc = vcs[s];
                double psi = q.w - phi_i;
#pragma unroll
                for (int a = 0; a < D; ++a) psi -= dx[a] * Gp[a];
                pair_sums<D, T>(r, T(vqs[s]), vc, T(psi), L2, acc);
                return;
            } else {
                pair_geom<D, KERNEL, T, true>(q, vj, xi, invR, dx, r, q2, vc, &iq4, use);
            }
            double psi = q.w - phi_i;
#pragma unroll
            for (int a = 0; a < D; ++a) psi -= dx[a] * Gp[a];
            pair_sums<D, T>(r, vc * iq4, vc, T(psi), L2, acc);
        };
        double4 qn = sd[cols(0)];
        T vn = sv[cols(0)];
#pragma unroll
        for (int s = 0; s < kS; ++s) {
            const double4 q = qn;
            const T vj = vn;
            if (s + 1 < kS) {
                qn = sd[cols(s + 1)];
                vn = sv[cols(s + 1)];
            }
            __builtin_amdgcn_sched_barrier(0);
            term2(q, vj, s < nslot, s);
            __builtin_amdgcn_sched_barrier(0);
        }
        for (int64_t e = tail + lane; e < re; e += kLanes) {
            const int t = col_at(e);
            term2(sd[t], sv[t], true, -1);
        }
        // epilogue: the group's sums to LDS, then one thread per (row, particle)
#pragma unroll
        for (int c = 0; c < nk; ++c) acc[c] = group_sum(acc[c], kLanes);
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < nk; ++c) sacc[pl][c] = acc[c];
        }
        __syncthreads();
        {
            const int q = threadIdx.x % kChunk;
            const int64_t iq = p0 + q;
            // the row index made opaque here, so that the state addresses are
            // formed now rather than kept in registers (or spilled) from the
            // start of the kernel
            int o0 = threadIdx.x / kChunk;
            asm volatile("" : "+v"(o0));
            if (iq < p1) {
                for (int o = o0; o < A.nrows; o += kThreads / kChunk)
                    A.out[((int64_t)f * n + iq) * A.nrows + o] =
                        out_row<D, T, S>(A, iq, o, &sacc[q][0], &sacc[q][nk]);
                if (GOUT && threadIdx.x < kChunk)
#pragma unroll
                    for (int a = 0; a < D; ++a) A.g_out[((int64_t)f * D + a) * n + iq] = (float)sacc[q][nk + a];
            }
        }
    }
}

template <int D, int KERNEL, class T, class S>
static int launch_apply(const ApplyArgs<S>& a, int64_t cap, hipStream_t s) {
    const dim3 grid((unsigned)cap), block(ApplyCfg<T>::threads);
    const char* name = sizeof(T) == 4 ? "k_apply (mixed)" : "k_apply (fp64)";
    if constexpr (!Scaled<T>::value) {
        if (a.g_in) {
            VCT_LAUNCH("k_apply (fp64, given G)", (k_apply<D, KERNEL, T, S, kGIn>), grid, block, 0, s, a);
            VCT_LAUNCH_CHECK();
            return VCT_OK;
        }
    }
    if (a.g_out)
        VCT_LAUNCH(name, (k_apply<D, KERNEL, T, S, kGOut>), grid, block, 0, s, a);
    else
        VCT_LAUNCH(name, (k_apply<D, KERNEL, T, S, kGNone>), grid, block, 0, s, a);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

template <class T, class S>
static int dispatch(int dim, int kernel, const ApplyArgs<S>& a, int64_t cap, hipStream_t s) {
    if (dim == 2)
        return kernel == VCT_KERNEL_WENDLAND_C2 ? launch_apply<2, VCT_KERNEL_WENDLAND_C2, T, S>(a, cap, s)
                                                : launch_apply<2, VCT_KERNEL_CUBIC_SPLINE, T, S>(a, cap, s);
    return kernel == VCT_KERNEL_WENDLAND_C2 ? launch_apply<3, VCT_KERNEL_WENDLAND_C2, T, S>(a, cap, s)
                                            : launch_apply<3, VCT_KERNEL_CUBIC_SPLINE, T, S>(a, cap, s);
}

template <class S>
static ApplyArgs<S> make_args(const vct_nlist* nl, const Grid& g, int nf, const double* phi, const double* pos,
                              const double* vol, const S* state, uint32_t mask, double* out) {
    const int dim = nl->dim;
    const int64_t ncols = dim == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    ApplyArgs<S> a;
    a.n = nl->n;
    a.nf = nf;
    a.nrows = n_out_rows(dim, mask);
    a.invR = 1.0 / nl->R;
    a.g = g;
    a.phi = phi;
    a.pos = pos;
    a.vol = vol;
    a.row_ptr = nl->row_ptr;
    a.col16 = nl->col16;
    a.cs = nl->cell_start;
    a.cstart = nl->chunk_start;
    a.cinfo = reinterpret_cast<const int4*>(nl->chunk_info); a.cwin = nl->chunk_win;
    a.nchunks = nl->chunk_off + ncols;
    a.state = state;
    a.out = out;
    a.g_out = nullptr;
    a.g_in = nullptr;
    return a;
}

VCT_CHECKS_TU(checks_apply)

}  // namespace vct

using namespace vct;

static int apply_ops(const vct_nlist* nl, int nf, const double* phi_sorted, const double* pos_sorted,
                     const double* vol_sorted, int kernel, const void* state, uint32_t out_mask, int precision,
                     double* out, float* g_out, const float* g_in, void* stream) {
    Grid g;
    int st = nlist_check(nl, g);
    if (st) return st;
    if (nf < 1 || !mask_valid(out_mask) ||
        (kernel != VCT_KERNEL_WENDLAND_C2 && kernel != VCT_KERNEL_CUBIC_SPLINE) ||
        (precision != VCT_FP64 && precision != VCT_MIXED && precision != VCT_MIXED_S64))
        return VCT_E_ARG;
    const int64_t n = nl->n;
    if (n == 0) return VCT_OK;
    if (!phi_sorted || !pos_sorted || !vol_sorted || !nl->col16 || !state || !out) return VCT_E_ARG;
    const int dim = nl->dim;
    const int64_t ncols = dim == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    const int64_t cap = ncols + n / kChunk + 1;   // upper bound of the chunk count
    hipStream_t s = as_stream(stream);
    switch (precision) {
    case VCT_FP64: {
        auto a = make_args(nl, g, nf, phi_sorted, pos_sorted, vol_sorted, static_cast<const double*>(state), out_mask,
                           out);
        a.g_out = g_out;
        a.g_in = g_in;
        return dispatch<double, double>(dim, kernel, a, cap, s);
    }
    case VCT_MIXED: {
        auto a = make_args(nl, g, nf, phi_sorted, pos_sorted, vol_sorted, static_cast<const float*>(state), out_mask,
                           out);
        a.g_out = g_out;
        return dispatch<float, float>(dim, kernel, a, cap, s);
    }
    default: {
        auto a = make_args(nl, g, nf, phi_sorted, pos_sorted, vol_sorted, static_cast<const double*>(state), out_mask,
                           out);
        a.g_out = g_out;
        return dispatch<float, double>(dim, kernel, a, cap, s);
    }
    }
}

extern "C" int vct_apply_ops(const vct_nlist* nl, int nf, const double* phi_sorted, const double* pos_sorted,
                             const double* vol_sorted, int kernel, const void* state, uint32_t out_mask,
                             int precision, double* out, void* stream) {
    VCT_API_RANGE("vct_apply_ops");
    return apply_ops(nl, nf, phi_sorted, pos_sorted, vol_sorted, kernel, state, out_mask, precision, out, nullptr,
                     nullptr, stream);
}

extern "C" int vct_apply_ops_ex(const vct_nlist* nl, int nf, const double* phi_sorted, const double* pos_sorted,
                                const double* vol_sorted, int kernel, const void* state, uint32_t out_mask,
                                int precision, double* out, float* g_out, const float* g_in, void* stream) {
    VCT_API_RANGE("vct_apply_ops_ex");
    if (g_out && g_in) return VCT_E_ARG;   // distinct roles: one call writes G~, a later one reads it
    return apply_ops(nl, nf, phi_sorted, pos_sorted, vol_sorted, kernel, state, out_mask, precision, out, g_out,
                     g_in, stream);
}
