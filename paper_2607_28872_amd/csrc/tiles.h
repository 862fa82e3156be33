// Column-aligned particle chunks and their LDS neighbour windows.
//
// The cell-sorted particles of one (x, y) cell column (2-D: one x column) are
// split into chunks of at most kChunk consecutive particles.  Every neighbour
// of a chunk's particles lies in the chunk's window: the 3^(d-1) columns
// around its own, restricted to the z cells spanned by the chunk widened by
// one cell on each side.  Each of those columns contributes one contiguous
// range of sorted indices, and the ranges are concatenated in increasing order
// of their first index.  A work-group stages the window's particle records in
// LDS once; neighbour lists stored as 16-bit window offsets then index LDS
// directly.  The window depends only on the grid, the cell table and the
// chunk, so the neighbour search and every consumer derive the same one.
#pragma once

#include "common.h"

namespace vct {

constexpr int kChunk = 64;        // particles per chunk
constexpr int kMaxRanges = 9;     // 3 x 3 columns in 3-D, 3 in 2-D

// Chunk table: chunk b covers sorted particles [start[b], start[b+1]) of
// column info[b].x, z cells [info[b].y, info[b].z].
struct ChunkTable {
    const int32_t* start;   // [nchunks + 1]
    const int4* info;       // [nchunks]: column, zlo, zhi, unused
    const int64_t* count;   // device scalar: number of chunks
};

template <int D> struct WindowT {
    int nr;
    int64_t gstart[kMaxRanges];
    int off[kMaxRanges + 1];
};

// Columns are numbered c0 * nc1 + c1 in 3-D and c0 in 2-D; z is the last axis.
template <int D>
__device__ __forceinline__ int64_t col_key(const Grid& g, int64_t col, int64_t z) {
    if (D == 3) return col * g.nc[2] + z;
    return col * g.nc[1] + z;
}

template <int D>
__device__ __forceinline__ int64_t grid_nz(const Grid& g) { return D == 3 ? g.nc[2] : g.nc[1]; }

template <int D>
__device__ __forceinline__ int64_t grid_ncols(const Grid& g) { return D == 3 ? g.nc[0] * g.nc[1] : g.nc[0]; }

// Window of a chunk (same result in every thread that calls it).
template <int D>
__device__ __forceinline__ void chunk_window(const Grid& g, const int64_t* __restrict__ cs, int4 info,
                                             WindowT<D>& w) {
    const int64_t nz = grid_nz<D>(g);
    const int64_t zlo = info.y > 0 ? info.y - 1 : 0;
    const int64_t zhi = info.z + 1 < nz ? info.z + 1 : nz - 1;
    int64_t cx, cy = 0;
    if (D == 3) { cx = info.x / g.nc[1]; cy = info.x % g.nc[1]; }
    else cx = info.x;
    w.nr = 0;
    int acc = 0;
    for (int dx = -1; dx <= 1; ++dx) {
        const int64_t x = cx + dx;
        if (x < 0 || x >= g.nc[0]) continue;
        for (int dy = (D == 3 ? -1 : 0); dy <= (D == 3 ? 1 : 0); ++dy) {
            int64_t colid;
            if (D == 3) {
                const int64_t y = cy + dy;
                if (y < 0 || y >= g.nc[1]) continue;
                colid = x * g.nc[1] + y;
            } else {
                colid = x;
            }
            const int64_t a = cs[col_key<D>(g, colid, zlo)], b = cs[col_key<D>(g, colid, zhi) + 1];
            w.gstart[w.nr] = a;
            w.off[w.nr] = acc;
            acc += (int)(b - a);
            ++w.nr;
        }
    }
    w.off[w.nr] = acc;
}

// The same window computed by one whole wave in parallel: lane r handles the
// r-th column of the 3^(d-1) (in the order of chunk_window), the ranges are
// compacted with a ballot and their offsets formed with a prefix sum over
// lanes.  Every lane of the calling wave must call it.
template <int D>
__device__ __forceinline__ void chunk_window_wave(const Grid& g, const int64_t* __restrict__ cs, int4 info,
                                                  WindowT<D>& w) {
    const int lane = threadIdx.x % kWave;
    const int64_t nz = grid_nz<D>(g);
    const int64_t zlo = info.y > 0 ? info.y - 1 : 0;
    const int64_t zhi = info.z + 1 < nz ? info.z + 1 : nz - 1;
    constexpr int ncand = D == 3 ? 9 : 3;
    int64_t x, y = 0, colid;
    if (D == 3) {
        x = info.x / g.nc[1] + lane / 3 - 1;
        y = info.x % g.nc[1] + lane % 3 - 1;
        colid = x * g.nc[1] + y;
    } else {
        x = info.x + lane - 1;
        colid = x;
    }
    const bool in = lane < ncand && x >= 0 && x < g.nc[0] && (D == 2 || (y >= 0 && y < g.nc[1]));
    int64_t a = 0;
    int len = 0;
    if (in) {
        a = cs[col_key<D>(g, colid, zlo)];
        len = (int)(cs[col_key<D>(g, colid, zhi) + 1] - a);
    }
    const uint64_t m = (uint64_t)__ballot(in);
    const int slot = __popcll(m & ((1ull << lane) - 1ull));
    int incl = len;
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
        const int v = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += v;
    }
    const int total = __shfl(incl, ncand - 1, kWave);
    if (in) {
        w.gstart[slot] = a;
        w.off[slot] = incl - len;
    }
    if (lane == 0) {
        w.nr = __popcll(m);
        w.off[__popcll(m)] = total;
    }
}

// Stored windows: chunk b's WindowT at tab + 32 b (int32 words).
static_assert(sizeof(WindowT<3>) <= 32 * sizeof(int32_t), "a stored window fits 32 words");
static_assert(sizeof(WindowT<2>) == sizeof(WindowT<3>), "one stored layout for both dimensions");

// Store (lanes 0..31 of the wave that formed w) or load (lanes 0..31 of any
// wave) a window as 32 int32 words.
template <int D>
__device__ __forceinline__ void window_store(const WindowT<D>& w, int32_t* __restrict__ tab, uint32_t b) {
    const int lane = threadIdx.x % kWave;
    if (lane < (int)(sizeof(WindowT<D>) / 4)) tab[(int64_t)b * 32 + lane] = reinterpret_cast<const int32_t*>(&w)[lane];
}
template <int D>
__device__ __forceinline__ void window_load(const int32_t* __restrict__ tab, uint32_t b, WindowT<D>& w) {
    const int lane = threadIdx.x % kWave;
    if (lane < (int)(sizeof(WindowT<D>) / 4)) reinterpret_cast<int32_t*>(&w)[lane] = tab[(int64_t)b * 32 + lane];
}

// global sorted index of window offset t
template <int D>
__device__ __forceinline__ int64_t window_global(const WindowT<D>& w, int t) {
    t = dcheck(t, w.off[w.nr], kChkWindow);
    int r = 0;
#pragma unroll
    for (int k = 1; k < kMaxRanges; ++k)
        if (k < w.nr && t >= w.off[k]) r = k;
    return w.gstart[r] + (t - w.off[r]);
}

}  // namespace vct
