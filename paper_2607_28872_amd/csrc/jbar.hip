// Volume smoothing of the sigma method: the smoothed Jacobian determinant
// Jbar^N of paper Sec. 3.6 (Eq. VCT_bar_a).
//
// With v_i = J_i / Jbar_i (particle i's representative volume in units of V),
// the update of one neighbour pair (i, j) in Eq. VCT_bar_a is a volume
// exchange:
//   c_ij = C_V (r_e - |r^_ij|) / r_e,   dv = c_ij (v_j - v_i),
//   v_i <- v_i + dv,   v_j <- v_j - dv,
// applied along the neighbours j of a target particle i one after the other,
// every exchange seen by the next, and then for the next target.  Every
// particle is a target once; the paper leaves the order of the targets open.
//
// Schedule.  The targets are taken cell by cell in 3^d phases: the cell
// (cx, [cy,] cz) belongs to phase (cx mod 3) + 3 (cy mod 3) + 9 (cz mod 3)
// (2-D: (cx mod 3) + 3 (cz mod 3)), phases in increasing order.  A target
// and its neighbours lie in the 3^d cells around the target's cell, and two
// cells of one phase are at least three cells apart along some axis, so those
// blocks of cells are disjoint and the cells of a phase are independent: one
// work-group per cell.  Within a cell the targets go in sorted order and the
// neighbours of each in the order of its row (ascending sorted index).  The
// result is the sequential definition with the targets ordered by (phase,
// cell, sorted index), up to rounding.
//
// Within one row the neighbours are distinct, so their values are read at
// once, and v_i after the first k exchanges is the composition of the affine
// maps x -> (1 - c_k) x + c_k v_jk: one prefix scan over the lanes (64
// entries at a time) gives v_i before every exchange, and with it every
// neighbour's new value (the scan runs on DPP row shifts and broadcasts).
// The v values of the cell's block are staged in LDS
// (blocks larger than the LDS area are updated in place in memory, the same
// arithmetic).  J / Jbar is formed once before the phases and J / v once
// after.
#include "common.h"
#include "map_dev.h"
#include "tiles.h"

namespace vct {

int nlist_check(const vct_nlist* nl, Grid& g);

constexpr int kJCap = 1024;   // block values staged in LDS (8 KB)

struct JbarArgs {
    int64_t n;
    Grid g;
    double cv, re;
    const double* pos;
    const int64_t* row_ptr;
    const uint16_t* col16;
    const int64_t* cs;
    const int64_t* chunk_off;
    const int32_t* cstart;
    const int4* cinfo;
    const int32_t* cwin;
    double* v;   // [n] J / Jbar, updated in place
};

__global__ __launch_bounds__(256) void k_jbar_ratio(int64_t n, const double* __restrict__ a,
                                                   const double* __restrict__ b, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] / b[i];
}

// position of sorted index i in a window (the range holding it), or -1
template <int D>
__device__ __forceinline__ int window_offset_of(const WindowT<D>& w, int64_t i) {
    int t = -1;
#pragma unroll
    for (int r = 0; r < kMaxRanges; ++r)
        if (r < w.nr && i >= w.gstart[r] && i < w.gstart[r] + (w.off[r + 1] - w.off[r]))
            t = w.off[r] + (int)(i - w.gstart[r]);
    return t;
}

// A 64-bit value moved across lanes by a DPP control (row shifts, row
// broadcasts, wave shift); lanes without a source, or masked by the row mask,
// keep `id`.
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ double dpp_move64(double v, double id) {
    const int lo = __builtin_amdgcn_update_dpp(__double2loint(id), __double2loint(v), CTRL, ROWMASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(__double2hiint(id), __double2hiint(v), CTRL, ROWMASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

// One step of the inclusive scan of affine maps x -> a x + b over the lanes
// (lane k composes its map after the one the control brings in; the identity
// (1, 0) for lanes without one leaves a and b exactly as they are).
template <int CTRL, int ROWMASK = 0xF>
__device__ __forceinline__ void affine_step(double& a, double& b) {
    const double ao = dpp_move64<CTRL, ROWMASK>(a, 1.0), bo = dpp_move64<CTRL, ROWMASK>(b, 0.0);
    b = fma(a, bo, b);
    a = a * ao;
}

// Inclusive scan over the 64 lanes: within rows of 16 by row shifts of 1, 2,
// 4 and 8, then row 0's total into row 1 (and row 2's into row 3) by the
// row-15 broadcast, then the first two rows' total into rows 2 and 3 by the
// row-31 broadcast.
__device__ __forceinline__ void affine_scan(double& a, double& b) {
    affine_step<0x111>(a, b);         // row_shr:1
    affine_step<0x112>(a, b);         // row_shr:2
    affine_step<0x114>(a, b);         // row_shr:4
    affine_step<0x118>(a, b);         // row_shr:8
    affine_step<0x142, 0xA>(a, b);    // row_bcast:15 into rows 1 and 3
    affine_step<0x143, 0xC>(a, b);    // row_bcast:31 into rows 2 and 3
}

constexpr int kJSlots = 2;   // row entries per lane taken together (rows of up to 128 in one pass)
constexpr int kJRows = 64;   // row pointers of a cell held in registers (longer cells reload them)

// Pair weights c = C_V (r_e - |r^_ij|) / r_e and value addresses of the
// entries [e0 + s 64 + lane] of one row (s < kJSlots), decoded through the
// window of the row's chunk; entries past `re` get c = 0 and no address.
template <int D>
__device__ __forceinline__ void row_geometry(const JbarArgs& A, const WindowT<D>& cw, const WindowT<D>& blk, bool fast,
                                             int64_t i, int64_t e0, int64_t re, double (&c)[kJSlots],
                                             int64_t (&jj)[kJSlots]) {
    const int lane = threadIdx.x;
    const int64_t n = A.n;
    double xi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xi[a] = a < D ? A.pos[a * n + i] : 0.0;
#pragma unroll
    for (int s = 0; s < kJSlots; ++s) {
        const int64_t e = e0 + s * kWave + lane;
        c[s] = 0.0;
        jj[s] = -1;
        if (e < re) {
            const int t = dcheck((int)A.col16[e], cw.off[cw.nr], kChkWindow);
            int r = 0;
#pragma unroll
            for (int k = 1; k < kMaxRanges; ++k)
                if (k < cw.nr && t >= cw.off[k]) r = k;
            const int64_t j = cw.gstart[r] + (t - cw.off[r]);
            // the chunk window and the block list the same columns in the same order
            jj[s] = fast ? blk.off[r] + (j - blk.gstart[r]) : j;
            double r2 = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const double d = A.pos[a * n + j] - xi[a];
                r2 += d * d;
            }
            c[s] = A.cv * (A.re - sqrt(r2)) / A.re;
        }
    }
}

// The exchanges of one cell (the body of k_jbar_phase).  FAST: the block's
// values are in LDS (vp = s_v, addressed by block offset); otherwise in
// memory (vp = A.v, addressed by sorted index).  The geometry of the next
// target's row (its window offsets and neighbour positions, which no exchange
// changes) is loaded while the current row's exchanges run.
template <int D, bool FAST>
__device__ __forceinline__ void jbar_cell(const JbarArgs& A, int64_t col, int64_t p0, int64_t p1, double* vp,
                                          const WindowT<D>& blk, WindowT<D> (&cw)[2]) {
    const int lane = threadIdx.x;
    const Grid& g = A.g;
    // row pointers of targets [q0, q0 + 63], lane k holding row_ptr[q0 + k]
    int64_t q0 = p0;
    int64_t rp = A.row_ptr[q0 + lane < p1 ? q0 + lane : p1];
    auto row_ptr_of = [&](int64_t i) {   // uniform i in [q0, q0 + kJRows)
        return __shfl(rp, (int)(i - q0), kWave);
    };
    // chunk of a target: the column's chunks in order
    int64_t bc = A.chunk_off[col];
    auto chunk_of = [&](int64_t i) {
        while (A.cstart[bc + 1] <= i) ++bc;
        return bc;
    };
    auto load_window = [&](int64_t chunk, WindowT<D>& w) {
        if (A.cwin) window_load<D>(A.cwin, (uint32_t)chunk, w);
        else chunk_window_wave<D>(g, A.cs, A.cinfo[chunk], w);
    };

    int cur = 0;
    int64_t bcur = chunk_of(p0);
    load_window(bcur, cw[cur]);
    __syncthreads();
    int64_t rb = row_ptr_of(p0), re = p0 + 1 - q0 < kJRows ? row_ptr_of(p0 + 1) : A.row_ptr[p0 + 1];
    double c[kJSlots];
    int64_t jj[kJSlots];
    row_geometry<D>(A, cw[cur], blk, FAST, p0, rb, re, c, jj);

    for (int64_t i = p0; i < p1; ++i) {
        // the next target's geometry first
        const bool more = i + 1 < p1;
        int64_t rb1 = 0, re1 = 0;
        int nxt = cur;
        double c1[kJSlots] = {};
        int64_t jj1[kJSlots] = {};
        if (more) {   // uniform
            if (i + 2 - q0 > kJRows) {   // refill the row pointers (uniform)
                q0 = i + 1;
                rp = A.row_ptr[q0 + lane < p1 ? q0 + lane : p1];
            }
            rb1 = row_ptr_of(i + 1);
            re1 = i + 2 - q0 < kJRows ? row_ptr_of(i + 2) : A.row_ptr[i + 2];
            const int64_t b1 = chunk_of(i + 1);
            if (b1 != bcur) {   // uniform: the next target starts a new chunk
                nxt = 1 - cur;
                load_window(b1, cw[nxt]);
                bcur = b1;
                __syncthreads();
            }
            row_geometry<D>(A, cw[nxt], blk, FAST, i + 1, rb1, re1, c1, jj1);
        }
        const int64_t ii = FAST ? window_offset_of<D>(blk, i) : i;
        double vi = vp[ii];
        for (int64_t e0 = rb; e0 < re; e0 += kWave * kJSlots) {
            if (e0 != rb) row_geometry<D>(A, cw[cur], blk, FAST, i, e0, re, c, jj);   // rows longer than 128
            double vj[kJSlots];
#pragma unroll
            for (int s = 0; s < kJSlots; ++s) vj[s] = jj[s] >= 0 ? vp[jj[s]] : 0.0;
            // slot by slot: the scan of the maps x -> (1 - c) x + c v_j gives
            // v_i before every lane's exchange (padding lanes are the identity)
#pragma unroll
            for (int s = 0; s < kJSlots; ++s) {
                double am = 1.0 - c[s], bm = c[s] * vj[s];
                affine_scan(am, bm);
                const double ap = dpp_move64<0x138>(am, 1.0), bp = dpp_move64<0x138>(bm, 0.0);   // wave_shr:1
                const double xk = fma(ap, vi, bp);
                if (jj[s] >= 0) vp[jj[s]] = vj[s] - c[s] * (vj[s] - xk);
                const double aT = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(am), kWave - 1),
                                                   __builtin_amdgcn_readlane(__double2loint(am), kWave - 1));
                const double bT = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(bm), kWave - 1),
                                                   __builtin_amdgcn_readlane(__double2loint(bm), kWave - 1));
                vi = fma(aT, vi, bT);
            }
        }
        if (lane == 0) vp[ii] = vi;
        __syncthreads();   // this row's values before the next row reads them
        cur = nxt;
        rb = rb1;
        re = re1;
#pragma unroll
        for (int s = 0; s < kJSlots; ++s) {
            c[s] = c1[s];
            jj[s] = jj1[s];
        }
    }
}

constexpr int kJWins = 4;   // chunk windows of one cell held in LDS on the pipelined path

// The exchanges of one cell whose block fits the LDS area and whose targets
// lie in at most kJWins chunks (whose windows are all in LDS, cwa[k] for
// chunk b0 + k, starting at sorted index cst[k]).  A three-stage pipeline
// over the targets: while target i's exchanges run, the neighbour positions
// of target i + 1 and the window offsets of target i + 2 are in flight (none
// of them depends on an exchange); the pair weights of i + 1 are formed after
// i's exchanges (the distance by the refined reciprocal square root, C_V / r_e
// formed once: the same weights to within an ulp).
template <int D>
__device__ __forceinline__ void jbar_cell_pipelined(const JbarArgs& A, int64_t p0, int64_t p1, double* s_v,
                                                    const WindowT<D>& blk, const WindowT<D>* cwa,
                                                    const int64_t (&cst)[kJWins], int nchk,
                                                    const int (*shl)[kMaxRanges], const int64_t (*shg)[kMaxRanges]) {
    const int lane = threadIdx.x;
    const int64_t n = A.n;
    const double cvr = A.cv / A.re;
    auto win_of = [&](int64_t i) {
        int k = 0;
#pragma unroll
        for (int q = 1; q < kJWins; ++q)
            if (q < nchk && i >= cst[q]) k = q;
        return k;
    };
    // row pointers of targets [q0, q0 + 63], lane k holding row_ptr[q0 + k];
    // queried for increasing targets only
    int64_t q0 = p0;
    int64_t rp = A.row_ptr[q0 + lane < p1 ? q0 + lane : p1];
    auto row_range = [&](int64_t i, int64_t& rb, int64_t& re) {   // uniform i < p1
        if (i + 1 - q0 >= kJRows) {
            q0 = i;
            rp = A.row_ptr[q0 + lane < p1 ? q0 + lane : p1];
        }
        rb = __shfl(rp, (int)(i - q0), kWave);
        re = __shfl(rp, (int)(i + 1 - q0), kWave);
    };
    // window offsets of the first kJSlots x 64 entries of a row (-1 past its end)
    auto load_offsets = [&](int64_t rb, int64_t re, int (&t)[kJSlots]) {
#pragma unroll
        for (int s = 0; s < kJSlots; ++s) {
            const int64_t e = rb + s * kWave + lane;
            t[s] = e < re ? (int)A.col16[e] : -1;
        }
    };
    // sorted index and block offset of window offset t of chunk window k:
    // its range r is the number of range starts at or below t, and each
    // range's two shifts are looked up in LDS
    auto decode = [&](int k, int t, int64_t& j, int64_t& jl) {
        const WindowT<D>& w = cwa[k];
        t = dcheck(t, w.off[w.nr], kChkWindow);
        int r = 0;
#pragma unroll
        for (int q = 1; q < kMaxRanges; ++q) r += (q < w.nr && t >= w.off[q]) ? 1 : 0;
        j = t + shg[k][r];
        jl = t + shl[k][r];
    };
    // neighbour positions of the decoded offsets (loads only) ...
    auto load_positions = [&](int k, const int (&t)[kJSlots], double (&xj)[kJSlots][3], int64_t (&jl)[kJSlots]) {
#pragma unroll
        for (int s = 0; s < kJSlots; ++s) {
            jl[s] = -1;
#pragma unroll
            for (int a = 0; a < 3; ++a) xj[s][a] = 0.0;
            if (t[s] >= 0) {
                int64_t j;
                decode(k, t[s], j, jl[s]);
#pragma unroll
                for (int a = 0; a < D; ++a) xj[s][a] = A.pos[a * n + j];
            }
        }
    };
    // ... and the pair weights c = C_V (r_e - |r^_ij|) / r_e from them
    auto weights = [&](const double (&xi)[3], const double (&xj)[kJSlots][3], const int64_t (&jl)[kJSlots],
                       double (&c)[kJSlots]) {
#pragma unroll
        for (int s = 0; s < kJSlots; ++s) {
            double r2 = 0.0;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const double d = xj[s][a] - xi[a];
                r2 += d * d;
            }
            c[s] = jl[s] >= 0 ? cvr * (A.re - vsqrt(r2)) : 0.0;
        }
    };
    auto target_pos = [&](int64_t i, double (&xi)[3]) {
#pragma unroll
        for (int a = 0; a < 3; ++a) xi[a] = a < D ? A.pos[a * n + i] : 0.0;
    };

    // prologue: target p0 complete, target p0 + 1's offsets
    int64_t rb, re, rb1 = 0, re1 = 0;
    row_range(p0, rb, re);
    double c[kJSlots], xi[3];
    int64_t jl[kJSlots];
    {
        int t0[kJSlots];
        double xj[kJSlots][3];
        load_offsets(rb, re, t0);
        load_positions(win_of(p0), t0, xj, jl);
        target_pos(p0, xi);
        weights(xi, xj, jl, c);
    }
    int t1[kJSlots] = {-1, -1};
    if (p0 + 1 < p1) {
        row_range(p0 + 1, rb1, re1);
        load_offsets(rb1, re1, t1);
    }

    for (int64_t i = p0; i < p1; ++i) {
        // in flight during i's exchanges: offsets of i + 2, positions of i + 1
        int64_t rb2 = 0, re2 = 0;
        int t2[kJSlots] = {-1, -1};
        if (i + 2 < p1) {   // uniform
            row_range(i + 2, rb2, re2);
            load_offsets(rb2, re2, t2);
        }
        double xj1[kJSlots][3], xi1[3] = {0.0, 0.0, 0.0};
        int64_t jl1[kJSlots] = {-1, -1};
        if (i + 1 < p1) {   // uniform
            load_positions(win_of(i + 1), t1, xj1, jl1);
            target_pos(i + 1, xi1);
        }

        // target i's exchanges
        const int ki = win_of(i);
        const int64_t ii = window_offset_of<D>(blk, i);
        double vi = s_v[ii];
        for (int64_t e0 = rb; e0 < re; e0 += kWave * kJSlots) {
            if (e0 != rb) {   // rows longer than kJSlots x 64 entries: the rest in place
                int tt[kJSlots];
                double xj[kJSlots][3];
                load_offsets(e0, re, tt);
                load_positions(ki, tt, xj, jl);
                weights(xi, xj, jl, c);
            }
            double vj[kJSlots];
#pragma unroll
            for (int s = 0; s < kJSlots; ++s) vj[s] = jl[s] >= 0 ? s_v[jl[s]] : 0.0;
            // slot by slot: the scan of the maps x -> (1 - c) x + c v_j gives
            // v_i before every lane's exchange (padding lanes are the identity)
#pragma unroll
            for (int s = 0; s < kJSlots; ++s) {
                double am = 1.0 - c[s], bm = c[s] * vj[s];
                affine_scan(am, bm);
                const double ap = dpp_move64<0x138>(am, 1.0), bp = dpp_move64<0x138>(bm, 0.0);   // wave_shr:1
                const double xk = fma(ap, vi, bp);
                if (jl[s] >= 0) s_v[jl[s]] = vj[s] - c[s] * (vj[s] - xk);
                const double aT = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(am), kWave - 1),
                                                   __builtin_amdgcn_readlane(__double2loint(am), kWave - 1));
                const double bT = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(bm), kWave - 1),
                                                   __builtin_amdgcn_readlane(__double2loint(bm), kWave - 1));
                vi = fma(aT, vi, bT);
            }
        }
        if (lane == 0) s_v[ii] = vi;
        __syncthreads();   // this row's values before the next row reads them

        // target i + 1's weights, then shift the pipeline
        if (i + 1 < p1) {   // uniform
#pragma unroll
            for (int a = 0; a < 3; ++a) xi[a] = xi1[a];
            weights(xi, xj1, jl1, c);
#pragma unroll
            for (int s = 0; s < kJSlots; ++s) {
                jl[s] = jl1[s];
                t1[s] = t2[s];
            }
            rb = rb1;
            re = re1;
            rb1 = rb2;
            re1 = re2;
        }
    }
}

// One cell of phase `phase` per work-group (one wave).
template <int D>
__global__ __launch_bounds__(kWave) void k_jbar_phase(JbarArgs A, int phase, int64_t uy, int64_t uz) {
    __shared__ double s_v[kJCap];
    __shared__ WindowT<D> blk;     // the 3^d cells around the cell
    __shared__ WindowT<D> cw[2];   // windows of the chunks of the current and the next target
    __shared__ WindowT<D> cwa[kJWins];   // windows of the cell's chunks (pipelined path)
    __shared__ int s_shl[kJWins][kMaxRanges];       // their offset -> block offset shifts
    __shared__ int64_t s_shg[kJWins][kMaxRanges];   // their offset -> sorted index shifts
    const int lane = threadIdx.x;
    const Grid& g = A.g;
    // the cell: z (last axis) fastest over the phase's cells
    int64_t b = blockIdx.x;
    int64_t cx, cy = 0, cz;
    if (D == 3) {
        cz = phase / 9 + 3 * (b % uz);
        b /= uz;
        cy = (phase / 3) % 3 + 3 * (b % uy);
        b /= uy;
        cx = phase % 3 + 3 * b;
    } else {
        cz = phase / 3 + 3 * (b % uz);
        b /= uz;
        cx = phase % 3 + 3 * b;
    }
    const int64_t col = D == 3 ? cx * g.nc[1] + cy : cx;
    const int64_t key = col_key<D>(g, col, cz);
    const int64_t p0 = A.cs[key], p1 = A.cs[key + 1];
    if (p0 == p1) return;   // uniform over the work-group
    chunk_window_wave<D>(g, A.cs, make_int4((int)col, (int)cz, (int)cz, 0), blk);
    __syncthreads();
    const int W = blk.off[blk.nr];
    if (W <= kJCap) {   // uniform
        for (int t = lane; t < W; t += kWave) s_v[t] = A.v[window_global<D>(blk, t)];
        // the chunks holding the cell's targets
        int64_t b0 = A.chunk_off[col];
        while (A.cstart[b0 + 1] <= p0) ++b0;
        int64_t bl = b0;
        while (A.cstart[bl + 1] < p1) ++bl;
        const int nchk = (int)(bl - b0 + 1);
        if (nchk <= kJWins) {   // uniform
            int64_t cst[kJWins];
#pragma unroll
            for (int k = 0; k < kJWins; ++k) {
                cst[k] = k < nchk ? (int64_t)A.cstart[b0 + k] : p1;
                if (k < nchk) {
                    if (A.cwin) window_load<D>(A.cwin, (uint32_t)(b0 + k), cwa[k]);
                    else chunk_window_wave<D>(g, A.cs, A.cinfo[b0 + k], cwa[k]);
                }
            }
            __syncthreads();
            // per window and range: window offset -> sorted index and -> block
            // offset (the chunk windows and the block list the same columns
            // in the same order)
            if (lane < nchk * kMaxRanges) {
                const int k = lane / kMaxRanges, r = lane % kMaxRanges;
                const WindowT<D>& w = cwa[k];
                const int64_t g0 = r < w.nr ? w.gstart[r] - w.off[r] : 0;
                s_shg[k][r] = g0;
                s_shl[k][r] = r < w.nr ? (int)(g0 - blk.gstart[r]) + blk.off[r] : 0;
            }
            __syncthreads();
            jbar_cell_pipelined<D>(A, p0, p1, s_v, blk, cwa, cst, nchk, s_shl, s_shg);
        } else {
            jbar_cell<D, true>(A, col, p0, p1, s_v, blk, cw);
        }
        __syncthreads();
        for (int t = lane; t < W; t += kWave) A.v[window_global<D>(blk, t)] = s_v[t];
    } else {
        jbar_cell<D, false>(A, col, p0, p1, A.v, blk, cw);
    }
}

// J = det J = alpha at every particle (Eq. det_jacobi)
__global__ __launch_bounds__(256) void k_map_alpha(int dim, int64_t n, const double* __restrict__ pos, MapParams mp,
                                                   double* __restrict__ alpha) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = pos[i], y = dim == 3 ? pos[n + i] : 0.0, zh = pos[(int64_t)(dim - 1) * n + i];
    alpha[i] = map_coef_at(mp, i, x, y, zh).alpha;
}

// projected positions of physical points: x^ = x, y^ = y, z^ = alpha (z + beta) (Eq. VCT)
__global__ __launch_bounds__(256) void k_map_project(int dim, int64_t n, const double* __restrict__ phys, MapParams mp,
                                                     double* __restrict__ proj) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = phys[i], y = dim == 3 ? phys[n + i] : 0.0, z = phys[(int64_t)(dim - 1) * n + i];
    const MapCoef<double> c = map_coef_at(mp, i, x, y, 0.0);
    for (int a = 0; a < dim - 1; ++a) proj[(int64_t)a * n + i] = phys[(int64_t)a * n + i];
    proj[(int64_t)(dim - 1) * n + i] = c.alpha * (z + c.beta);
}

VCT_CHECKS_TU(checks_jbar)

}  // namespace vct

using namespace vct;

extern "C" size_t vct_jbar_workspace_size(int64_t n) {
    if (n < 0) return 0;
    return aligned_sum({(size_t)(n > 0 ? n : 1) * sizeof(double)});
}

extern "C" int vct_jbar_smooth(const vct_nlist* nl, const double* pos_sorted, const double* J, double* jbar, double cv,
                               double re, void* ws, size_t ws_bytes, void* stream) {
    VCT_API_RANGE("vct_jbar_smooth");
    Grid g;
    int st = nlist_check(nl, g);
    if (st) return st;
    if (!isfinite(cv) || !(re > 0.0) || !isfinite(re)) return VCT_E_ARG;
    const int64_t n = nl->n;
    if (n == 0) return VCT_OK;
    if (!pos_sorted || !J || !jbar || !nl->col16) return VCT_E_ARG;
    if (!ws || ws_bytes < vct_jbar_workspace_size(n)) return VCT_E_WORKSPACE;
    Carver cv_ws(ws, ws_bytes);
    double* v = cv_ws.take<double>((size_t)n);
    hipStream_t s = as_stream(stream);
    JbarArgs a;
    a.n = n; a.g = g; a.cv = cv; a.re = re; a.pos = pos_sorted; a.row_ptr = nl->row_ptr; a.col16 = nl->col16;
    a.cs = nl->cell_start; a.chunk_off = nl->chunk_off; a.cstart = nl->chunk_start;
    a.cinfo = reinterpret_cast<const int4*>(nl->chunk_info); a.cwin = nl->chunk_win; a.v = v;
    const unsigned nb = (unsigned)((n + 255) / 256);
    VCT_LAUNCH("k_jbar_ratio", k_jbar_ratio, dim3(nb), dim3(256), 0, s, n, J, jbar, v);
    VCT_LAUNCH_CHECK();
    const int dim = nl->dim;
    const int nph = dim == 3 ? 27 : 9;
    const int64_t nx = g.nc[0], ny = dim == 3 ? g.nc[1] : 1, nz = dim == 3 ? g.nc[2] : g.nc[1];
    auto count = [](int64_t nc, int64_t p) { return nc > p ? (nc - p + 2) / 3 : 0; };
    for (int ph = 0; ph < nph; ++ph) {
        const int64_t ux = count(nx, ph % 3);
        const int64_t uy = dim == 3 ? count(ny, (ph / 3) % 3) : 1;
        const int64_t uz = count(nz, dim == 3 ? ph / 9 : ph / 3);
        const int64_t cells = ux * uy * uz;
        if (cells == 0) continue;
        if (dim == 3) VCT_LAUNCH("k_jbar_phase", k_jbar_phase<3>, dim3((unsigned)cells), dim3(kWave), 0, s, a, ph, uy, uz);
        else VCT_LAUNCH("k_jbar_phase", k_jbar_phase<2>, dim3((unsigned)cells), dim3(kWave), 0, s, a, ph, uy, uz);
        VCT_LAUNCH_CHECK();
    }
    VCT_LAUNCH("k_jbar_ratio", k_jbar_ratio, dim3(nb), dim3(256), 0, s, n, J, v, jbar);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

extern "C" int vct_map_alpha(int dim, int64_t n, const double* pos, const vct_map* map, double* alpha, void* stream) {
    VCT_API_RANGE("vct_map_alpha");
    if ((dim != 2 && dim != 3) || n < 0 || !map) return VCT_E_ARG;
    MapParams mp;
    const int st = map_params_from(map, dim, n, mp);
    if (st) return st;
    if (n == 0) return VCT_OK;
    if (!pos || !alpha) return VCT_E_ARG;
    VCT_LAUNCH("k_map_alpha", k_map_alpha, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream), dim, n,
               pos, mp, alpha);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

extern "C" int vct_map_project(int dim, int64_t n, const double* phys, const vct_map* map, double* proj, void* stream) {
    VCT_API_RANGE("vct_map_project");
    if ((dim != 2 && dim != 3) || n < 0 || !map) return VCT_E_ARG;
    MapParams mp;
    const int st = map_params_from(map, dim, n, mp);
    if (st) return st;
    if (n == 0) return VCT_OK;
    if (!phys || !proj || phys == proj) return VCT_E_ARG;
    VCT_LAUNCH("k_map_project", k_map_project, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream),
               dim, n, phys, mp, proj);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}
