// Background-cell sort and neighbour lists (paper Sec. 3.1, Eq. SPH_neighbor_set;
// neighbour searches with background cells, Sec. 3.4).
//
// Cells are at least R wide, so every neighbour of a particle lies in the
// 3^d cells around its own.  Particles are sorted by (cell key, original index)
// with a counting sort; z is the fastest cell axis, so the three z-adjacent
// cells of one (x, y) column are contiguous in memory and each particle's
// candidates form 3^(d-1) contiguous ranges, visited in increasing order.
#include "common.h"
#include "tiles.h"

namespace vct {

// ------------------------------------------------------------------ small kernels

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static int fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return VCT_OK;
    VCT_LAUNCH("k_fill_i32", k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

static int fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s) {
    if (n <= 0) return VCT_OK;
    VCT_LAUNCH("k_fill_i64", k_fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

// ------------------------------------------------------------------ exclusive scan

// out[i] = sum_{k<i} in[k] for i in [0, n], int32 -> int64, in three passes:
// per-tile sums, a single-block scan of the tile sums, per-tile scans.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ int64_t block_exclusive_scan(int64_t v, int64_t* lds_waves, int64_t* total) {
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    int64_t inc = v;
    for (int o = 1; o < kWave; o <<= 1) {
        int64_t t = __shfl_up(inc, o, kWave);
        if (lane >= o) inc += t;
    }
    if (lane == kWave - 1) lds_waves[wv] = inc;
    __syncthreads();
    int64_t wbase = 0, tot = 0;
    for (int k = 0; k < kScanThreads / kWave; ++k) {
        if (k < wv) wbase += lds_waves[k];
        tot += lds_waves[k];
    }
    __syncthreads();
    *total = tot;
    return wbase + inc - v;
}

__global__ void k_scan_tiles(const int32_t* in, int64_t n, int64_t* tile_sums) {
    __shared__ int64_t lw[kScanThreads / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k)
        if (base + k < n) s += in[base + k];
    int64_t tot;
    block_exclusive_scan(s, lw, &tot);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ void k_scan_sums(int64_t* sums, int64_t ntiles, int64_t* out_total) {
    __shared__ int64_t lw[kScanThreads / kWave];
    int64_t carry = 0;
    for (int64_t b = 0; b < ntiles; b += kScanThreads) {
        int64_t i = b + threadIdx.x;
        int64_t v = i < ntiles ? sums[i] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_scan(v, lw, &tot);
        if (i < ntiles) sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *out_total = carry;
}

__global__ void k_scan_apply(const int32_t* in, int64_t n, const int64_t* tile_off, int64_t* out) {
    __shared__ int64_t lw[kScanThreads / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    int64_t tot;
    int64_t run = tile_off[blockIdx.x] + block_exclusive_scan(s, lw, &tot);
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

static size_t scan_ws_bytes(int64_t n) {
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    return (size_t)(ntiles > 0 ? ntiles : 1) * sizeof(int64_t);
}

// out has n + 1 entries; out[n] is the total
static int exclusive_scan(const int32_t* in, int64_t n, int64_t* out, int64_t* tile_ws, hipStream_t s) {
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ntiles == 0) return fill_i64(out, 1, 0, s);
    VCT_LAUNCH("k_scan_tiles", k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in, n, tile_ws);
    VCT_LAUNCH_CHECK();
    VCT_LAUNCH("k_scan_sums", k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, tile_ws, ntiles, out + n);
    VCT_LAUNCH_CHECK();
    VCT_LAUNCH("k_scan_apply", k_scan_apply, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in, n, tile_ws, out);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

// ------------------------------------------------------------------ cell sort

// The key of every particle, and its slot in its cell (the count the atomic
// increment returns; the slots of a cell are a permutation of 0..count-1 in
// an order that varies from run to run, which the per-cell sort removes).
__global__ void k_cell_keys(int dim, int64_t n, const double* __restrict__ pos, Grid g,
                            int32_t* __restrict__ keys, int32_t* __restrict__ slots,
                            int32_t* __restrict__ counts, int32_t* __restrict__ bad) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t c[3] = {0, 0, 0};
    bool finite = true;
    for (int a = 0; a < dim; ++a) {
        double v = pos[a * n + i];
        finite = finite && isfinite(v);
        c[a] = cell_coord(v, g.lo[a], g.inv_cs[a], g.nc[a]);
    }
    if (!finite) atomicAdd(bad, 1);
    int32_t k = (int32_t)cell_key(c[0], c[1], c[2], g);
    keys[i] = k;
    slots[i] = atomicAdd(&counts[k], 1);
}

__global__ void k_cell_scatter(int64_t n, const int32_t* __restrict__ keys, const int32_t* __restrict__ slots,
                               const int64_t* __restrict__ cell_start, int32_t* __restrict__ perm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    perm[cell_start[keys[i]] + slots[i]] = (int32_t)i;
}

// The scatter leaves each cell's particles in arbitrary order; sorting every
// cell's slice by original index makes the result deterministic.  A slice of
// at most kSortReg entries is sorted in registers by a bitonic network (the
// slots past its end hold INT_MAX and stay at the end); a longer one by
// insertion in place.
constexpr int kSortReg = 64;
__global__ void k_cell_sort(int64_t ncell, const int64_t* __restrict__ cell_start,
                            int32_t* __restrict__ perm) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int64_t b = cell_start[c], e = cell_start[c + 1];
    if (e - b <= kSortReg) {
        const int len = (int)(e - b);
        int v[kSortReg];
#pragma unroll
        for (int k = 0; k < kSortReg; ++k) v[k] = k < len ? perm[b + k] : INT_MAX;
#pragma unroll
        for (int size = 2; size <= kSortReg; size <<= 1)
#pragma unroll
            for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
                for (int k = 0; k < kSortReg; ++k) {
                    const int l = k ^ stride;
                    if (l > k) {
                        const bool up = (k & size) == 0;   // ascending half
                        const int lo = v[k] < v[l] ? v[k] : v[l], hi = v[k] < v[l] ? v[l] : v[k];
                        v[k] = up ? lo : hi;
                        v[l] = up ? hi : lo;
                    }
                }
#pragma unroll
        for (int k = 0; k < kSortReg; ++k)
            if (k < len) perm[b + k] = v[k];
        return;
    }
    for (int64_t i = b + 1; i < e; ++i) {
        int32_t v = perm[i];
        int64_t j = i - 1;
        while (j >= b && perm[j] > v) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = v;
    }
}

// Components move in groups of four whose loads are all issued before the
// first store: the scattered side then costs one memory latency per group,
// not one per component.
__global__ void k_gather(int64_t n, int ncomp, const int32_t* __restrict__ perm,
                         const double* __restrict__ src, double* __restrict__ dst) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t o = perm[s];
    for (int c0 = 0; c0 < ncomp; c0 += 4) {
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (c0 + k < ncomp) v[k] = src[(c0 + k) * n + o];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (c0 + k < ncomp) dst[(c0 + k) * n + s] = v[k];
    }
}

__global__ void k_scatter(int64_t n, int ncomp, const int32_t* __restrict__ perm,
                          const double* __restrict__ src, double* __restrict__ dst) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t o = perm[s];
    for (int c0 = 0; c0 < ncomp; c0 += 4) {
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (c0 + k < ncomp) v[k] = src[(c0 + k) * n + s];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (c0 + k < ncomp) dst[(c0 + k) * n + o] = v[k];
    }
}

// ------------------------------------------------------------------ chunk table

// Chunks of one column: ceil(count / kChunk) pieces of consecutive particles.
template <int D>
__global__ void k_chunk_count(Grid g, const int64_t* __restrict__ cs, int32_t* __restrict__ nch) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= grid_ncols<D>(g)) return;
    const int64_t nz = grid_nz<D>(g);
    const int64_t cnt = cs[col_key<D>(g, c, nz - 1) + 1] - cs[col_key<D>(g, c, 0)];
    nch[c] = (int32_t)((cnt + kChunk - 1) / kChunk);
}

// z cell of sorted particle p inside column c (largest z with cs[key(c, z)] <= p)
template <int D>
__device__ int64_t z_of(const Grid& g, const int64_t* __restrict__ cs, int64_t c, int64_t p) {
    int64_t lo = 0, hi = grid_nz<D>(g) - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (cs[col_key<D>(g, c, mid)] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int D>
__global__ void k_chunk_fill(Grid g, int64_t n, const int64_t* __restrict__ cs, const int64_t* __restrict__ off,
                             int32_t* __restrict__ cstart, int4* __restrict__ cinfo) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ncols = grid_ncols<D>(g);
    if (c >= ncols) {
        if (c == ncols) cstart[off[ncols]] = (int32_t)n;
        return;
    }
    const int64_t nz = grid_nz<D>(g);
    const int64_t a = cs[col_key<D>(g, c, 0)], e = cs[col_key<D>(g, c, nz - 1) + 1];
    int64_t b = off[c];
    for (int64_t p = a; p < e; p += kChunk, ++b) {
        const int64_t q = (p + kChunk < e ? p + kChunk : e) - 1;
        cstart[b] = (int32_t)p;
        cinfo[b] = make_int4((int)c, (int)z_of<D>(g, cs, c, p), (int)z_of<D>(g, cs, c, q), 0);
    }
}

// ------------------------------------------------------------------ neighbours

// The neighbour test of Eq. SPH_neighbor_set: d2 summed left to right in FP64
// with no fused multiply-add (so the sets are reproducible bit for bit).
__device__ __forceinline__ bool within_exact(double dx, double dy, double dz, double R2) {
#pragma clang fp contract(off)
    double d2 = dx * dx;
    d2 = d2 + dy * dy;
    d2 = d2 + dz * dz;
    return d2 < R2;
}

// d2 - lim for an FP32 window record q (offset from the chunk origin, with
// |q|^2 in q.w) and the particle's FP32 offset f, expanded as
// |q|^2 + (|f|^2 - lim) - 2 q . f: c = |f|^2 - lim and m = -2 f per
// particle, so a candidate costs one add and three multiply-adds.  The
// expansion's rounding grows with the offsets' size M instead of with d2
// (bound below, where the band is set).
__device__ __forceinline__ float d2_minus(const float4& q, float m0, float m1, float m2, float c) {
    return fmaf(q.x, m0, fmaf(q.y, m1, fmaf(q.z, m2, q.w + c)));
}

constexpr int kNbWaves = 4;                    // waves per work-group
constexpr int kNbThreads = kNbWaves * kWave;   // one chunk per work-group, lane = particle
constexpr int kNbSeg = 1536;                   // window records per LDS segment (24 KB)
constexpr int kNbWords = kNbSeg / 32;          // 32-candidate words per segment
constexpr int kStage = 128;                    // 16-bit staging slots per particle in the workspace
constexpr int kBmWords = kStage / 2;           // hit words per particle slot: windows up to 2048 candidates

// One chunk per work-group; every wave holds the whole chunk, lane = particle,
// and takes a quarter of the window's candidates.  The window is staged in
// LDS segment by segment as FP32 offsets from the chunk's first particle; all
// lanes of a wave test the same candidate (one broadcast LDS read), so a test
// costs a few VALU instructions.  A candidate whose FP32 squared distance is
// inside or outside R^2 by more than a bound on its rounding error is decided
// by it; the few near the support edge are re-tested with the exact FP64
// predicate on the stored positions.  Hits are collected as one bit per
// candidate (32-candidate words).
// MODE 0 writes the counts.  MODE 1 writes the columns at row_ptr (sorted
// indices and/or 16-bit window offsets): the words go to LDS ([word][particle])
// and a per-particle prefix over the waves' hit counts places every wave's
// hits, in ascending window order, in the particle's row.  MODE 2 writes the
// counts and the chunk's hit words, [word][particle] with the chunk's np
// particles per word, at word p0 * kBmWords of `col16` (the staging buffer),
// for k_nb_expand to turn into rows; a window wider than kBmWords * 32
// candidates does not fit there and is flagged (overflow[2]).  overflow[0]
// flags windows beyond 65535.
template <int D, int MODE>
__global__ __launch_bounds__(kNbThreads) void k_nb_chunk(int64_t n, const double* __restrict__ pos, Grid g,
                                                         double R2, const int64_t* __restrict__ cs,
                                                         const int32_t* __restrict__ cstart,
                                                         const int4* __restrict__ cinfo,
                                                         const int64_t* __restrict__ nchunks,
                                                         int32_t* __restrict__ counts,
                                                         const int64_t* __restrict__ row_ptr,
                                                         int32_t* __restrict__ col, uint16_t* __restrict__ col16,
                                                         int32_t* __restrict__ overflow,
                                                         int32_t* __restrict__ win_tab) {
    constexpr bool FILL = MODE == 1, STAGE = MODE == 2;
    static_assert(kChunk == kWave, "lane = particle");
    static_assert(kNbSeg % 32 == 0, "segments hold whole words");
    __shared__ float4 win[kNbSeg];
    __shared__ uint32_t bm[FILL ? kNbWords : 1][kChunk];
    __shared__ int32_t wcnt[kNbWaves][kChunk];
    __shared__ float wmax[kNbWaves];
    __shared__ WindowT<D> w;
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *nchunks) return;   // uniform over the work-group
    const int64_t p0 = cstart[b], p1 = cstart[b + 1];
    const int np = (int)(p1 - p0);
    const int wv = threadIdx.x / kWave, pl = threadIdx.x % kWave;
    if (wv == 0) chunk_window_wave<D>(g, cs, cinfo[b], w);
    const int64_t i = p0 + pl;
    const bool valid = pl < np;
    const int64_t ii = valid ? i : p0;
    // the chunk origin: its middle particle, which keeps the offsets (and the
    // rounding of the expanded distance) small
    const int64_t pm = p0 + (np - 1) / 2;
    const double o0 = pos[pm], o1 = pos[n + pm], o2 = (D == 3) ? pos[2 * n + pm] : 0.0;
    const double xi0 = pos[ii], xi1 = pos[n + ii], xi2 = (D == 3) ? pos[2 * n + ii] : 0.0;
    // offsets from the chunk origin in FP32 (the same rounding as the records)
    const float f0 = (float)(xi0 - o0), f1 = (float)(xi1 - o1), f2 = (float)(xi2 - o2);
    const float fmax_own = fmaxf(fabsf(f0), fmaxf(fabsf(f1), fabsf(f2)));
    const float m0 = -2.0f * f0, m1 = -2.0f * f1, m2 = -2.0f * f2;   // exact
    const float ff = fmaf(f2, f2, fmaf(f1, f1, f0 * f0));
    const int64_t rlo = FILL ? row_ptr[ii] : 0, rlen = FILL ? row_ptr[ii + 1] - rlo : 0;
    __syncthreads();
    const int W = w.off[w.nr];
    if ((FILL || STAGE) && threadIdx.x == 0 && W > 65535) atomicOr(overflow, 1);
    if (win_tab && wv == 0) window_store<D>(w, win_tab, b);   // for the later calls
    // the particle's own window offset (it is never its own neighbour)
    int self_t = -1;
    for (int r = 0; r < w.nr; ++r) {
        const int64_t d = i - w.gstart[r];
        if (d >= 0 && d < w.off[r + 1] - w.off[r]) self_t = w.off[r] + (int)d;
    }
    // the chunk's hit words (MODE 2), np per word; only when they fit its
    // share of the staging buffer (np * kBmWords words)
    const bool bm_fit = W <= kBmWords * 32;
    if (STAGE && threadIdx.x == 0 && !bm_fit) atomicOr(overflow + 2, 1);
    uint32_t* bmg = STAGE && bm_fit ? reinterpret_cast<uint32_t*>(col16) + p0 * kBmWords : nullptr;
    int rowpos = 0;                     // entries of the row found so far (MODE 1)
    int mycnt = 0;                      // hits of this wave's candidates (MODES 0, 2)
    for (int s0 = 0; s0 < W; s0 += kNbSeg) {
        const int sW = W - s0 < kNbSeg ? W - s0 : kNbSeg;
        if (s0 > 0) __syncthreads();   // the previous segment is consumed
        // stage the segment: every load of a thread before its first LDS store
        {
            constexpr int kRep = kNbSeg / kNbThreads;
            double px[kRep], py[kRep], pz[kRep];
#pragma unroll
            for (int k = 0; k < kRep; ++k) {
                const int t = threadIdx.x + k * kNbThreads;
                const int64_t j = window_global<D>(w, s0 + (t < sW ? t : 0));
                px[k] = pos[j];
                py[k] = pos[n + j];
                pz[k] = D == 3 ? pos[2 * n + j] : 0.0;
            }
            float mo = 0.0f;
#pragma unroll
            for (int k = 0; k < kRep; ++k) {
                const int t = threadIdx.x + k * kNbThreads;
                if (t < sW) {
                    float4 q = make_float4((float)(px[k] - o0), (float)(py[k] - o1),
                                           D == 3 ? (float)(pz[k] - o2) : 0.0f, 0.0f);
                    q.w = fmaf(q.z, q.z, fmaf(q.y, q.y, q.x * q.x));
                    win[t] = q;
                    mo = fmaxf(mo, fmaxf(fabsf(q.x), fmaxf(fabsf(q.y), fabsf(q.z))));
                }
            }
#pragma unroll
            for (int m = kWave / 2; m >= 1; m >>= 1) mo = fmaxf(mo, __shfl_xor(mo, m, kWave));
            if (pl == 0) wmax[wv] = mo;
        }
        __syncthreads();
        // Absolute bound on the FP32 error of t against the exact d2 - R^2,
        // with M the largest offset component (staged or own) and u = 2^-24:
        // the rounded offsets, |d2(q, f) - d2| <= 4 sqrt(3) u M |q - f| <=
        // 24 u M^2; the three roundings of each of |q|^2 and |f|^2 (3 u
        // 3M^2 each), the rounding of |f|^2 - lim, of the add and of the three
        // multiply-adds, each relative to a partial result below 12 M^2 + R^2
        // (57 u M^2 + 5 u R^2 in all); and the rounding of lim to FP32 (u R^2).
        // 96 u M^2 + 8 u R^2 covers the sum.
        const float mseg = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
        const double maxoff = (double)fmaxf(mseg, fmax_own);
        const double margin = (96.0 * maxoff * maxoff + 8.0 * R2) * 0x1p-24;
        const float in_lim = (float)(R2 - margin), out_lim = (float)(R2 + margin);
        const float cf = ff - in_lim;
        // t = d2 - in_lim: t < 0 is a certain hit, 0 <= t <= band is the
        // uncertain band (as unsigned integers, exactly the non-negative t up
        // to band: a negative t has its sign bit set), t > band certainly
        // lies outside.  band = out_lim - in_lim, rounded up if the FP32
        // difference is inexact (offsets beyond about 240 R).
        const double band_d = (double)out_lim - (double)in_lim;   // exact in FP64
        float band = (float)band_d;
        if ((double)band < band_d) band = nextafterf(band, INFINITY);
        const uint32_t band_u = __float_as_uint(band);
        const int nw = (sW + 31) / 32;
        const int k0 = wv * nw / kNbWaves, k1 = (wv + 1) * nw / kNbWaves;
        [[maybe_unused]] int cnt = 0;   // this segment's hits of this wave (MODE 1)
        for (int k = k0; k < k1; ++k) {
            // Hits shift in as the sign bits of t (the first candidate ends in
            // bit 31, reversed below); whether any candidate of the word lies
            // in the band is one flag per lane, rarely set.
            uint32_t bits = 0u;
            bool amb_any = false;
            const float4* wp = win + 32 * k;
            // records read eight at a time, the next eight while the current
            // ones are tested
            float4 rec[8], nxt[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) rec[u] = wp[u];   // same record, every lane
#pragma unroll
            for (int u0 = 0; u0 < 32; u0 += 8) {
                if (u0 + 8 < 32) {
#pragma unroll
                    for (int u = 0; u < 8; ++u) nxt[u] = wp[u0 + 8 + u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const uint32_t t = __float_as_uint(d2_minus(rec[u], m0, m1, m2, cf));
                    bits = __builtin_amdgcn_alignbit(bits, t, 31);
                    amb_any = amb_any || t <= band_u;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) rec[u] = nxt[u];
            }
            bits = __builtin_bitreverse32(bits);
            // drop the tail beyond the segment, the particle itself, idle lanes
            const int tb = s0 + 32 * k;
            uint32_t keep = (sW - 32 * k) >= 32 ? 0xffffffffu : ((1u << (sW - 32 * k)) - 1u);
            if (self_t >= tb && self_t < tb + 32) keep &= ~(1u << (self_t - tb));
            if (!valid) keep = 0u;
            bits &= keep;
            if (amb_any) {
                // the word's candidates in the band, from the same arithmetic
                // (the empty asm keeps the compiler from carrying the t of the
                // loop above over to here), then the exact FP64 predicate
                float g0 = m0, g1 = m1, g2 = m2, gc = cf;
                asm volatile("" : "+v"(g0), "+v"(g1), "+v"(g2), "+v"(gc));
                uint32_t amb = 0u;
#pragma unroll 1
                for (int u = 0; u < 32; ++u)
                    if (__float_as_uint(d2_minus(wp[u], g0, g1, g2, gc)) <= band_u) amb |= 1u << u;
                amb &= keep;
                while (amb) {
                    const int u = __builtin_ctz(amb);
                    amb &= amb - 1u;
                    const int64_t j = window_global<D>(w, tb + u);
                    if (within_exact(pos[j] - xi0, pos[n + j] - xi1, D == 3 ? pos[2 * n + j] - xi2 : 0.0, R2))
                        bits |= 1u << u;
                }
            }
            if constexpr (FILL) {
                bm[k][pl] = bits;
                cnt += __popc(bits);
            } else {
                if (STAGE && bmg && valid)
                    bmg[dcheck((s0 / 32 + k) * np + pl, np * kBmWords, kChkCapacity)] = bits;
                mycnt += __popc(bits);
            }
        }
        // MODES 0 and 2 sum the counts once, after the last segment
        if constexpr (FILL) {
            wcnt[wv][pl] = cnt;
            __syncthreads();
            // place this wave's hits after those of the earlier waves
            int pos0 = rowpos, total = 0;
#pragma unroll
            for (int v = 0; v < kNbWaves; ++v) {
                const int c = wcnt[v][pl];
                if (v < wv) pos0 += c;
                total += c;
            }
            if (valid) {
                int at = pos0;
                for (int k = k0; k < k1; ++k) {
                    uint32_t bits = bm[k][pl];
                    while (bits) {
                        const int t = s0 + 32 * k + __builtin_ctz(bits);
                        bits &= bits - 1u;
                        if (at < rlen) {
                            if (col) col[rlo + at] = (int32_t)window_global<D>(w, t);
                            if (col16) col16[rlo + at] = (uint16_t)t;
                        }
                        ++at;
                    }
                }
            }
            rowpos += total;
        }
    }
    if constexpr (!FILL) {
        wcnt[wv][pl] = mycnt;
        __syncthreads();
        if (wv == 0 && valid) {
            int c = 0;
#pragma unroll
            for (int v = 0; v < kNbWaves; ++v) c += wcnt[v][pl];
            counts[i] = c;
        }
    }
}

// Turn every chunk's hit words (written by k_nb_chunk in MODE 2) into its
// rows behind row_ptr: 16-bit window offsets, and sorted indices through the
// chunk window when col is wanted.  The words are [word][particle], np
// particles per word.  Lane = particle, and the eight waves take an eighth of
// the words each: every non-empty (word, particle) gets its first output
// position (the row's start, the earlier waves' share of the row, the hits
// before the word) and goes into a list ordered by its number of hits (a
// counting sort in LDS).  Taken in that order, the lanes of a wave expand
// words with about the same number of hits, so the loop over a word's bits
// does not wait for the fullest word of 64.  The positions are fixed before
// the expansion, so its order does not matter.  A list entry is 4 bytes (the
// particle, the word and the hits of the row before it; the word's bits are
// read again from the L2), which keeps the LDS at four work-groups per CU.
// The entries go to the chunk's block in LDS, which the work-group stores
// with unit stride; a chunk whose block exceeds the LDS buffer writes its
// entries to memory directly.
constexpr int kExT = 512;                     // threads of k_nb_expand
constexpr int kExOut = 8192;                  // entries of a chunk's block in LDS (16 KB)
constexpr int kExList = kBmWords * kChunk;    // every (word, particle) of a chunk can be listed (16 KB)
template <int D>
__global__ __launch_bounds__(kExT) void k_nb_expand(Grid g, const int64_t* __restrict__ cs,
                                                    const int32_t* __restrict__ cstart,
                                                    const int4* __restrict__ cinfo,
                                                    const int64_t* __restrict__ nchunks,
                                                    const int64_t* __restrict__ row_ptr,
                                                    const uint32_t* __restrict__ words,
                                                    const int32_t* __restrict__ win_tab,
                                                    int32_t* __restrict__ col, uint16_t* __restrict__ col16) {
    constexpr int kWaves = kExT / kWave;
    constexpr int kPer = kBmWords / kWaves;   // words of one wave's share
    static_assert(kBmWords % kWaves == 0 && kChunk == kWave, "shares of whole words, lane = particle");
    __shared__ WindowT<D> w;
    __shared__ int64_t rp[kChunk + 1];
    __shared__ int32_t part[kWaves][kChunk];      // each wave's share of every row
    __shared__ uint32_t bucket[33];               // words per hit count (32 - count), then offsets
    __shared__ uint32_t list[kExList];            // particle | word << 6 | hits of the row before it << 12
    __shared__ uint16_t sout[kExOut];
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *nchunks) return;   // uniform over the work-group
    const int64_t p0 = cstart[b];
    const int np = (int)(cstart[b + 1] - p0);
    const int wv = threadIdx.x / kWave, pl = threadIdx.x % kWave;
    const uint32_t* src = words + p0 * kBmWords;
    const int k0 = wv * kPer;
    const bool lane_on = pl < np;
    // this wave's share of the words, requested with the window and the row
    // pointers: all kBmWords words of the chunk's share of the buffer (np x
    // kBmWords), those past the window (not written by the search) masked
    // once the window is known
    uint32_t v[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) v[u] = lane_on ? src[(k0 + u) * np + pl] : 0u;
    if (wv == 0) {
        if (win_tab) window_load<D>(win_tab, b, w);
        else chunk_window_wave<D>(g, cs, cinfo[b], w);
    }
    if (threadIdx.x <= (unsigned)np) rp[threadIdx.x] = row_ptr[p0 + threadIdx.x];
    if (threadIdx.x < 33) bucket[threadIdx.x] = 0u;
    __syncthreads();
    // at most kBmWords words: the search flags wider windows, and the host
    // then runs the fill pass instead
    const int nw = dcheck((w.off[w.nr] + 31) / 32, kBmWords + 1, kChkCapacity);
    const int64_t e0 = rp[0], e1 = rp[np];
    int before[kPer];   // hits of the row in this wave's share before each word
    {
#pragma unroll
        for (int u = 0; u < kPer; ++u) v[u] = k0 + u < nw ? v[u] : 0u;
        int c = 0;
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            before[u] = c;
            c += __popc(v[u]);
        }
        part[wv][pl] = c;
    }
    __syncthreads();
    int start = 0;   // hits of the row in the earlier waves' shares
    for (int x = 0; x < wv; ++x) start += part[x][pl];
    uint32_t slot[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) slot[u] = v[u] ? atomicAdd(&bucket[32 - __popc(v[u])], 1u) : 0u;
    __syncthreads();
    if (wv == 0) {   // exclusive prefix of the 32 bucket sizes; bucket[32] = the total
        const uint32_t t = pl < 32 ? bucket[pl] : 0u;
        uint32_t incl = t;
#pragma unroll
        for (int m = 1; m < 64; m <<= 1) {
            const uint32_t o = __shfl_up(incl, m, kWave);
            if (pl >= m) incl += o;
        }
        if (pl <= 32) bucket[pl] = incl - t;
    }
    __syncthreads();
    const int nlist = (int)bucket[32];   // the non-empty words (words without hits are not listed)
#pragma unroll
    for (int u = 0; u < kPer; ++u)
        if (v[u])
            list[dcheck((int)(bucket[32 - __popc(v[u])] + slot[u]), kExList, kChkCapacity)] =
                (uint32_t)pl | ((uint32_t)(k0 + u) << 6) | ((uint32_t)(start + before[u]) << 12);
    __syncthreads();
    const bool in_lds = e1 - e0 <= kExOut;
    auto expand = [&](uint32_t bits, int at, int wd) {
        while (bits) {
            const uint16_t t = (uint16_t)(32 * wd + __builtin_ctz(bits));
            bits &= bits - 1u;
            if (in_lds) {
                sout[dcheck(at, kExOut, kChkCapacity)] = t;
            } else {
                if (col16) col16[e0 + at] = t;
                if (col) col[e0 + at] = (int32_t)window_global<D>(w, t);
            }
            ++at;
        }
    };
    for (int li = threadIdx.x; li < nlist; li += kExT) {
        const uint32_t ent = list[li];
        const int q = (int)(ent & 63u), wd = (int)((ent >> 6) & 63u);
        expand(src[wd * np + q], (int)(rp[q] - e0) + (int)(ent >> 12), wd);
    }
    if (!in_lds) return;   // uniform over the work-group
    __syncthreads();
    for (int e = threadIdx.x; e < (int)(e1 - e0); e += kExT) {
        const uint16_t t = sout[e];
        if (col16) col16[e0 + e] = t;
        if (col) col[e0 + e] = (int32_t)window_global<D>(w, t);
    }
}

VCT_CHECKS_TU(checks_cells)

}  // namespace vct

using namespace vct;

// ====================================================================== C ABI

extern "C" int64_t vct_grid_dims(int dim, const double* lo, const double* hi, double R, int64_t* dims) {
    if ((dim != 2 && dim != 3) || !lo || !hi || !(R > 0.0) || !isfinite(R)) return VCT_E_ARG;
    Grid g;
    int64_t total = grid_setup(dim, lo, hi, R, g);
    if (total < 0) return total;
    if (dims) for (int a = 0; a < 3; ++a) dims[a] = g.nc[a];
    return total;
}

extern "C" size_t vct_build_cells_workspace_size(int dim, int64_t n, int64_t ncell) {
    (void)dim;
    if (n < 0 || ncell < 1) return 0;
    return aligned_sum({(size_t)n * 4, (size_t)n * 4, (size_t)ncell * 4, scan_ws_bytes(ncell), 64});
}

extern "C" int vct_build_cells(int dim, int64_t n, const double* pos, const double* lo, const double* hi,
                               double R, int32_t* perm, double* pos_sorted, int64_t* cell_start,
                               int64_t ncell, void* ws, size_t ws_bytes, void* stream) {
    VCT_API_RANGE("vct_build_cells");
    if ((dim != 2 && dim != 3) || n < 0 || n > INT32_MAX || !lo || !hi || !(R > 0.0) || !isfinite(R))
        return VCT_E_ARG;
    Grid g;
    int64_t total = grid_setup(dim, lo, hi, R, g);
    if (total < 0) return (int)total;
    if (ncell != total || !cell_start) return VCT_E_ARG;
    if (n > 0 && (!pos || !perm || !pos_sorted)) return VCT_E_ARG;
    if (!ws || ws_bytes < vct_build_cells_workspace_size(dim, n, ncell)) return VCT_E_WORKSPACE;
    hipStream_t s = as_stream(stream);
    Carver cv(ws, ws_bytes);
    int32_t* keys = cv.take<int32_t>((size_t)n);
    int32_t* slots = cv.take<int32_t>((size_t)n);
    int32_t* counts = cv.take<int32_t>((size_t)ncell);
    int64_t* tiles = cv.take<int64_t>(scan_ws_bytes(ncell) / 8);
    int32_t* bad = cv.take<int32_t>(16);
    int st;
    if ((st = fill_i32(counts, ncell, 0, s))) return st;
    if ((st = fill_i32(bad, 1, 0, s))) return st;
    if (n > 0) {
        VCT_LAUNCH("k_cell_keys", k_cell_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dim, n, pos, g,
                   keys, slots, counts, bad);
        VCT_LAUNCH_CHECK();
    }
    if ((st = exclusive_scan(counts, ncell, cell_start, tiles, s))) return st;
    if (n > 0) {
        VCT_LAUNCH("k_cell_scatter", k_cell_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, keys,
                   slots, cell_start, perm);
        VCT_LAUNCH_CHECK();
        VCT_LAUNCH("k_cell_sort", k_cell_sort, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, ncell,
                   cell_start, perm);
        VCT_LAUNCH_CHECK();
        VCT_LAUNCH("k_gather", k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, dim, perm, pos,
                   pos_sorted);
        VCT_LAUNCH_CHECK();
    }
    int32_t hbad = 0;
    VCT_HIP_CHECK(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VCT_HIP_CHECK(hipStreamSynchronize(s));
    return hbad ? VCT_E_NONFINITE : VCT_OK;
}

extern "C" int vct_gather_sorted(int64_t n, int ncomp, const int32_t* perm, const double* src, double* dst,
                                 void* stream) {
    VCT_API_RANGE("vct_gather_sorted");
    if (n < 0 || ncomp < 1 || n > INT32_MAX) return VCT_E_ARG;
    if (n == 0) return VCT_OK;
    if (!perm || !src || !dst || src == dst) return VCT_E_ARG;
    VCT_LAUNCH("k_gather", k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream), n, ncomp,
               perm, src, dst);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

extern "C" int vct_scatter_sorted(int64_t n, int ncomp, const int32_t* perm, const double* src, double* dst,
                                  void* stream) {
    VCT_API_RANGE("vct_scatter_sorted");
    if (n < 0 || ncomp < 1 || n > INT32_MAX) return VCT_E_ARG;
    if (n == 0) return VCT_OK;
    if (!perm || !src || !dst || src == dst) return VCT_E_ARG;
    VCT_LAUNCH("k_scatter", k_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream), n, ncomp,
               perm, src, dst);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

extern "C" int64_t vct_chunk_capacity(int dim, int64_t n, int64_t ncell) {
    if ((dim != 2 && dim != 3) || n < 0 || ncell < 1) return 0;
    return n / kChunk + ncell + 1;
}

// Workspace without the staging buffer (enough for the two-pass search).
static size_t nb_ws_base(int64_t n, int64_t ncell) {
    const int64_t m = n > ncell ? n : ncell;
    return aligned_sum({(size_t)m * 4, scan_ws_bytes(m), 64});
}

extern "C" size_t vct_neighbors_workspace_size(int64_t n, int64_t ncell) {
    if (n < 0 || ncell < 1) return 0;
    return aligned_sum({nb_ws_base(n, ncell), (size_t)(n > 0 ? n : 1) * kStage * sizeof(uint16_t)});
}

namespace vct {
// Transposed-entry map: for entry e = (i, j) of row i, the position of (j, i)
// in row j, found by binary search of i in row j's ascending columns.  The
// neighbour relation is symmetric (d2 is formed from x_j - x_i, whose
// negation is exact), so every search succeeds; a miss raises the flag.
// Each lane holds kTSlots entries and advances all their searches together,
// so the dependent loads of one step are in flight at once.
constexpr int kTLanes = 8;
constexpr int kTSlots = 16;
__global__ __launch_bounds__(256) void k_col_transpose(int64_t n, const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col, int32_t* __restrict__ col_t,
                                                       int32_t* __restrict__ miss) {
    // consecutive particles on one XCD: the rows a search reads are those of
    // nearby particles, which then stay in that XCD's L2
    const int64_t blk = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t i = (blk * blockDim.x + threadIdx.x) / kTLanes;
    const int lane = threadIdx.x % kTLanes;
    if (i >= n) return;
    const int64_t rb = row_ptr[i], re = row_ptr[i + 1];
    for (int64_t e0 = rb + lane; e0 < re; e0 += (int64_t)kTLanes * kTSlots) {
        int64_t lo[kTSlots], hi[kTSlots];
        bool act[kTSlots];
#pragma unroll
        for (int s = 0; s < kTSlots; ++s) {
            const int64_t e = e0 + (int64_t)kTLanes * s;
            act[s] = e < re;
            const int64_t j = act[s] ? col[e] : i;
            lo[s] = row_ptr[j];
            hi[s] = row_ptr[j + 1] - 1;
        }
        bool more = true;
        while (more) {
            more = false;
            int32_t v[kTSlots];
#pragma unroll
            for (int s = 0; s < kTSlots; ++s) {
                const bool go = act[s] && lo[s] < hi[s];
                v[s] = go ? col[(lo[s] + hi[s]) / 2] : 0;
            }
#pragma unroll
            for (int s = 0; s < kTSlots; ++s) {
                if (act[s] && lo[s] < hi[s]) {
                    const int64_t mid = (lo[s] + hi[s]) / 2;
                    if (v[s] < i) lo[s] = mid + 1;
                    else hi[s] = mid;
                    more = more || lo[s] < hi[s];
                }
            }
        }
#pragma unroll
        for (int s = 0; s < kTSlots; ++s) {
            const int64_t e = e0 + (int64_t)kTLanes * s;
            if (act[s]) {
                const bool ok = lo[s] <= hi[s] && col[lo[s]] == (int32_t)i;
                col_t[e] = ok ? (int32_t)lo[s] : -1;
                if (!ok) atomicOr(miss, 1);
            }
        }
    }
}

int nlist_check(const vct_nlist* nl, Grid& g) {
    if (!nl || (nl->dim != 2 && nl->dim != 3) || nl->n < 0 || nl->n > INT32_MAX || !(nl->R > 0.0) ||
        !isfinite(nl->R) || !nl->cell_start || !nl->row_ptr || !nl->chunk_off || !nl->chunk_start ||
        !nl->chunk_info || (reinterpret_cast<uintptr_t>(nl->col16) & 15u) != 0)
        return VCT_E_ARG;
    const int64_t total = grid_setup(nl->dim, nl->lo, nl->hi, nl->R, g);
    if (total < 0) return (int)total;
    if (total != nl->ncell || nl->chunk_cap < vct_chunk_capacity(nl->dim, nl->n, nl->ncell)) return VCT_E_ARG;
    return VCT_OK;
}
}  // namespace vct

template <int D>
static int build_chunks(const vct_nlist* nl, const Grid& g, int32_t* tmp, int64_t* tiles, hipStream_t s) {
    const int64_t ncols = D == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    const unsigned nb = (unsigned)((ncols + 1 + 255) / 256);
    VCT_LAUNCH("k_chunk_count", (k_chunk_count<D>), dim3(nb), dim3(256), 0, s, g, nl->cell_start, tmp);
    VCT_LAUNCH_CHECK();
    int st = exclusive_scan(tmp, ncols, nl->chunk_off, tiles, s);
    if (st) return st;
    VCT_LAUNCH("k_chunk_fill", (k_chunk_fill<D>), dim3(nb), dim3(256), 0, s, g, nl->n, nl->cell_start, nl->chunk_off,
               nl->chunk_start, reinterpret_cast<int4*>(nl->chunk_info));
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

template <int D, int MODE>
static int launch_nb(const vct_nlist* nl, const double* pos, const Grid& g, int32_t* counts, int32_t* overflow,
                     uint16_t* staged, hipStream_t s) {
    const int64_t ncols = D == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    const int64_t cap = ncols + nl->n / kChunk + 1;   // upper bound of the chunk count
    const char* name = MODE == 0 ? "k_nb_chunk (count)" : MODE == 1 ? "k_nb_chunk (fill)" : "k_nb_chunk (stage)";
    VCT_LAUNCH(name, (k_nb_chunk<D, MODE>), dim3((unsigned)cap), dim3(kNbThreads), 0, s, nl->n, pos, g,
               nl->R * nl->R, nl->cell_start, nl->chunk_start,
               reinterpret_cast<const int4*>(nl->chunk_info), nl->chunk_off + ncols, counts, nl->row_ptr,
               MODE == 1 ? nl->col : nullptr, MODE == 1 ? nl->col16 : staged, overflow, nl->chunk_win);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

template <int D>
static int launch_expand(const vct_nlist* nl, const Grid& g, const uint16_t* staged, hipStream_t s) {
    const int64_t ncols = D == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    const int64_t cap = ncols + nl->n / kChunk + 1;
    VCT_LAUNCH("k_nb_expand", (k_nb_expand<D>), dim3((unsigned)cap), dim3(kExT), 0, s, g, nl->cell_start,
               nl->chunk_start, reinterpret_cast<const int4*>(nl->chunk_info), nl->chunk_off + ncols,
               nl->row_ptr, reinterpret_cast<const uint32_t*>(staged), nl->chunk_win, nl->col, nl->col16);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

extern "C" int vct_neighbors(vct_nlist* nl, const double* pos_sorted, int64_t col_cap, int64_t* nnz_out,
                             int reuse_row_ptr, void* ws, size_t ws_bytes, void* stream) {
    VCT_API_RANGE("vct_neighbors");
    Grid g;
    int st = nlist_check(nl, g);
    if (st) return st;
    if (!nnz_out || (nl->n > 0 && !pos_sorted)) return VCT_E_ARG;
    const int64_t n = nl->n;
    if (!ws || ws_bytes < vct_neighbors_workspace_size(n, nl->ncell)) return VCT_E_WORKSPACE;
    hipStream_t s = as_stream(stream);
    Carver cv(ws, ws_bytes);
    const int64_t m = n > nl->ncell ? n : nl->ncell;
    int32_t* counts = cv.take<int32_t>((size_t)m);
    int64_t* tiles = cv.take<int64_t>(scan_ws_bytes(m) / 8);
    int32_t* flag = cv.take<int32_t>(16);
    uint16_t* staged = cv.take<uint16_t>((size_t)(n > 0 ? n : 1) * kStage);
    const int D = nl->dim;
    const bool want_cols = nl->col || nl->col16;
    // flag[0]: window wider than 16-bit offsets; flag[1]: transpose miss;
    // flag[2]: a window whose hit words exceed the staging capacity
    if ((st = fill_i32(flag, 3, 0, s))) return st;
    bool staged_ok = false;
    if (!reuse_row_ptr) {
        st = (D == 2) ? build_chunks<2>(nl, g, counts, tiles, s) : build_chunks<3>(nl, g, counts, tiles, s);
        if (st) return st;
        if (n > 0) {
            if (want_cols)
                st = (D == 2) ? launch_nb<2, 2>(nl, pos_sorted, g, counts, flag, staged, s)
                              : launch_nb<3, 2>(nl, pos_sorted, g, counts, flag, staged, s);
            else
                st = (D == 2) ? launch_nb<2, 0>(nl, pos_sorted, g, counts, flag, nullptr, s)
                              : launch_nb<3, 0>(nl, pos_sorted, g, counts, flag, nullptr, s);
            if (st) return st;
        }
        if ((st = exclusive_scan(counts, n, nl->row_ptr, tiles, s))) return st;
        staged_ok = want_cols;
    }
    int64_t nnz = 0;
    int32_t hflag[3] = {0, 0, 0};
    VCT_HIP_CHECK(hipMemcpyAsync(&nnz, nl->row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    VCT_HIP_CHECK(hipMemcpyAsync(hflag, flag, 3 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VCT_HIP_CHECK(hipStreamSynchronize(s));
    *nnz_out = nnz;
    nl->nnz = nnz;
    if (!want_cols) return VCT_OK;
    if (col_cap < nnz) return VCT_E_CAPACITY;
    if (nl->col_t && (!nl->col || nnz > INT32_MAX)) return VCT_E_ARG;
    if (hflag[0]) return VCT_E_WINDOW;
    if (n > 0) {
        if (staged_ok && !hflag[2])
            st = (D == 2) ? launch_expand<2>(nl, g, staged, s) : launch_expand<3>(nl, g, staged, s);
        else   // a window too wide for the staged hit words, or row_ptr given: the fill pass
            st = (D == 2) ? launch_nb<2, 1>(nl, pos_sorted, g, nullptr, flag, nullptr, s)
                          : launch_nb<3, 1>(nl, pos_sorted, g, nullptr, flag, nullptr, s);
        if (st) return st;
    }
    if (nl->col_t && n > 0) {
        VCT_LAUNCH("k_col_transpose", k_col_transpose, dim3((unsigned)((n * kTLanes + 255) / 256)), dim3(256), 0, s, n,
                   nl->row_ptr, nl->col, nl->col_t, flag + 1);
        VCT_LAUNCH_CHECK();
    }
    VCT_HIP_CHECK(hipMemcpyAsync(hflag, flag, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VCT_HIP_CHECK(hipStreamSynchronize(s));
    if (hflag[0]) return VCT_E_WINDOW;
    return hflag[1] ? VCT_E_HIP : VCT_OK;
}
