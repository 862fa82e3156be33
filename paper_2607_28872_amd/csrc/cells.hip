// Background-cell sort and neighbour lists (paper Sec. 3.1, Eq. SPH_neighbor_set;
// neighbour searches with background cells, Sec. 3.4).
//
// Cells are at least R wide, so every neighbour of a particle lies in the
// 3^d cells around its own.  Particles are sorted by (cell key, original index)
// with a counting sort; z is the fastest cell axis, so the three z-adjacent
// cells of one (x, y) column are contiguous in memory and each particle's
// candidates form 3^(d-1) contiguous ranges, visited in increasing order.
#include "common.h"

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
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

static int fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s) {
    if (n <= 0) return VCT_OK;
    hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
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
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in, n, tile_ws);
    VCT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, tile_ws, ntiles, out + n);
    VCT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)ntiles), dim3(kScanThreads), 0, s, in, n, tile_ws, out);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

// ------------------------------------------------------------------ cell sort

__global__ void k_cell_keys(int dim, int64_t n, const double* __restrict__ pos, Grid g,
                            int32_t* __restrict__ keys, int32_t* __restrict__ counts,
                            int32_t* __restrict__ bad) {
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
    atomicAdd(&counts[k], 1);
}

__global__ void k_cell_scatter(int64_t n, const int32_t* __restrict__ keys,
                               const int64_t* __restrict__ cell_start, int32_t* __restrict__ fill,
                               int32_t* __restrict__ perm) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t k = keys[i];
    int32_t slot = atomicAdd(&fill[k], 1);
    perm[cell_start[k] + slot] = (int32_t)i;
}

// The scatter leaves each cell's particles in arbitrary order; sorting every
// cell's slice by original index makes the result deterministic.
__global__ void k_cell_sort(int64_t ncell, const int64_t* __restrict__ cell_start,
                            int32_t* __restrict__ perm) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    int64_t b = cell_start[c], e = cell_start[c + 1];
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

__global__ void k_gather(int64_t n, int ncomp, const int32_t* __restrict__ perm,
                         const double* __restrict__ src, double* __restrict__ dst) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t o = perm[s];
    for (int c = 0; c < ncomp; ++c) dst[c * n + s] = src[c * n + o];
}

__global__ void k_scatter(int64_t n, int ncomp, const int32_t* __restrict__ perm,
                          const double* __restrict__ src, double* __restrict__ dst) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int64_t o = perm[s];
    for (int c = 0; c < ncomp; ++c) dst[c * n + o] = src[c * n + s];
}

// ------------------------------------------------------------------ neighbours

// The neighbour test of Eq. SPH_neighbor_set: d2 summed left to right in FP64
// with no fused multiply-add (so the sets are reproducible bit for bit).
template <int D>
__device__ __forceinline__ bool within(const double* __restrict__ pos, int64_t n, int64_t i, int64_t j,
                                       double xi0, double xi1, double xi2, double R2) {
#pragma clang fp contract(off)
    double dx = pos[j] - xi0;
    double dy = pos[n + j] - xi1;
    double d2 = dx * dx;
    d2 = d2 + dy * dy;
    if (D == 3) {
        double dz = pos[2 * n + j] - xi2;
        d2 = d2 + dz * dz;
    }
    return d2 < R2 && j != i;
}

// One group of G lanes per particle.  FILL = false counts, FILL = true writes
// the columns in ascending order (ballot compaction within the group).
template <int D, int G, bool FILL>
__global__ __launch_bounds__(256) void k_neighbors(int64_t n, const double* __restrict__ pos, Grid g,
                                                   double R2, const int64_t* __restrict__ cell_start,
                                                   int32_t* __restrict__ counts,
                                                   const int64_t* __restrict__ row_ptr,
                                                   int32_t* __restrict__ col) {
    constexpr int PER_BLOCK = 256 / G;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x % G;
    const int64_t i = (int64_t)tile * PER_BLOCK + threadIdx.x / G;
    const int gshift = (threadIdx.x % kWave) / G * G;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << gshift);
    const uint64_t below = (1ull << (threadIdx.x % kWave)) - 1ull;
    if (i >= n) return;   // whole groups exit together
    const double xi0 = pos[i], xi1 = pos[n + i], xi2 = (D == 3) ? pos[2 * n + i] : 0.0;
    int64_t c0 = cell_coord(xi0, g.lo[0], g.inv_cs[0], g.nc[0]);
    int64_t c1 = cell_coord(xi1, g.lo[1], g.inv_cs[1], g.nc[1]);
    int64_t c2 = (D == 3) ? cell_coord(xi2, g.lo[2], g.inv_cs[2], g.nc[2]) : 0;
    int64_t written = 0;
    const int64_t out0 = FILL ? row_ptr[i] : 0;
    const int64_t out1 = FILL ? row_ptr[i + 1] : 0;   // writes never pass the row end
    // 2-D: axes (x, z) -> cells (c0, c1), z fastest; 3-D: (c0, c1, c2), z fastest
    const int64_t a_lo = c0 > 0 ? c0 - 1 : 0, a_hi = c0 + 1 < g.nc[0] ? c0 + 1 : g.nc[0] - 1;
    const int64_t b_lo = (D == 3) ? (c1 > 0 ? c1 - 1 : 0) : 0;
    const int64_t b_hi = (D == 3) ? (c1 + 1 < g.nc[1] ? c1 + 1 : g.nc[1] - 1) : 0;
    const int64_t zc = (D == 3) ? c2 : c1;
    const int64_t nz = (D == 3) ? g.nc[2] : g.nc[1];
    const int64_t z_lo = zc > 0 ? zc - 1 : 0, z_hi = zc + 1 < nz ? zc + 1 : nz - 1;
    for (int64_t a = a_lo; a <= a_hi; ++a) {
        for (int64_t b = b_lo; b <= b_hi; ++b) {
            int64_t k_lo = (D == 3) ? cell_key(a, b, z_lo, g) : cell_key(a, z_lo, 0, g);
            int64_t k_hi = (D == 3) ? cell_key(a, b, z_hi, g) : cell_key(a, z_hi, 0, g);
            const int64_t jb = cell_start[k_lo], je = cell_start[k_hi + 1];
            for (int64_t base = jb; base < je; base += G) {
                const int64_t j = base + lane;
                const bool hit = (j < je) && within<D>(pos, n, i, j, xi0, xi1, xi2, R2);
                const uint64_t m = (uint64_t)__ballot(hit) & gmask;
                if (FILL && hit) {
                    const int64_t at = out0 + written + __popcll(m & below);
                    if (at < out1) col[at] = (int32_t)j;
                }
                written += __popcll(m);
            }
        }
    }
    if (!FILL && lane == 0) counts[i] = (int32_t)written;
}

template <int D, int G, bool FILL>
static int launch_neighbors(int64_t n, const double* pos, const Grid& g, double R2,
                            const int64_t* cell_start, int32_t* counts, const int64_t* row_ptr,
                            int32_t* col, hipStream_t s) {
    constexpr int PER_BLOCK = 256 / G;
    int64_t nb = (n + PER_BLOCK - 1) / PER_BLOCK;
    hipLaunchKernelGGL((k_neighbors<D, G, FILL>), dim3((unsigned)nb), dim3(256), 0, s, n, pos, g, R2,
                       cell_start, counts, row_ptr, col);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

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
    return aligned_sum({(size_t)n * 4, (size_t)ncell * 4, scan_ws_bytes(ncell), 64});
}

extern "C" int vct_build_cells(int dim, int64_t n, const double* pos, const double* lo, const double* hi,
                               double R, int32_t* perm, double* pos_sorted, int64_t* cell_start,
                               int64_t ncell, void* ws, size_t ws_bytes, void* stream) {
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
    int32_t* counts = cv.take<int32_t>((size_t)ncell);
    int64_t* tiles = cv.take<int64_t>(scan_ws_bytes(ncell) / 8);
    int32_t* bad = cv.take<int32_t>(16);
    int st;
    if ((st = fill_i32(counts, ncell, 0, s))) return st;
    if ((st = fill_i32(bad, 1, 0, s))) return st;
    if (n > 0) {
        hipLaunchKernelGGL(k_cell_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dim, n, pos, g,
                           keys, counts, bad);
        VCT_LAUNCH_CHECK();
    }
    if ((st = exclusive_scan(counts, ncell, cell_start, tiles, s))) return st;
    if (n > 0) {
        if ((st = fill_i32(counts, ncell, 0, s))) return st;
        hipLaunchKernelGGL(k_cell_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, keys,
                           cell_start, counts, perm);
        VCT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_cell_sort, dim3((unsigned)((ncell + 255) / 256)), dim3(256), 0, s, ncell,
                           cell_start, perm);
        VCT_LAUNCH_CHECK();
        hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, dim, perm, pos,
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
    if (n < 0 || ncomp < 1 || n > INT32_MAX) return VCT_E_ARG;
    if (n == 0) return VCT_OK;
    if (!perm || !src || !dst || src == dst) return VCT_E_ARG;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream), n, ncomp,
                       perm, src, dst);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

extern "C" int vct_scatter_sorted(int64_t n, int ncomp, const int32_t* perm, const double* src, double* dst,
                                  void* stream) {
    if (n < 0 || ncomp < 1 || n > INT32_MAX) return VCT_E_ARG;
    if (n == 0) return VCT_OK;
    if (!perm || !src || !dst || src == dst) return VCT_E_ARG;
    hipLaunchKernelGGL(k_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, as_stream(stream), n, ncomp,
                       perm, src, dst);
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

extern "C" size_t vct_neighbors_workspace_size(int64_t n) {
    if (n < 0) return 0;
    return aligned_sum({(size_t)n * 4, scan_ws_bytes(n), 64});
}

extern "C" int vct_neighbors(int dim, int64_t n, const double* pos_sorted, const double* lo, const double* hi,
                             double R, const int64_t* cell_start, int64_t ncell, int64_t* row_ptr,
                             int32_t* col, int64_t col_cap, int64_t* nnz_out, int reuse_row_ptr, void* ws,
                             size_t ws_bytes, void* stream) {
    if ((dim != 2 && dim != 3) || n < 0 || n > INT32_MAX || !lo || !hi || !(R > 0.0) || !isfinite(R) ||
        !row_ptr || !nnz_out || !cell_start)
        return VCT_E_ARG;
    Grid g;
    int64_t total = grid_setup(dim, lo, hi, R, g);
    if (total < 0) return (int)total;
    if (ncell != total) return VCT_E_ARG;
    if (n > 0 && !pos_sorted) return VCT_E_ARG;
    if (!ws || ws_bytes < vct_neighbors_workspace_size(n)) return VCT_E_WORKSPACE;
    hipStream_t s = as_stream(stream);
    Carver cv(ws, ws_bytes);
    int32_t* counts = cv.take<int32_t>((size_t)n);
    int64_t* tiles = cv.take<int64_t>(scan_ws_bytes(n) / 8);
    const double R2 = R * R;
    int st;
    if (!reuse_row_ptr) {
        if (n > 0) {
            st = (dim == 2) ? launch_neighbors<2, 16, false>(n, pos_sorted, g, R2, cell_start, counts, nullptr,
                                                             nullptr, s)
                            : launch_neighbors<3, 64, false>(n, pos_sorted, g, R2, cell_start, counts, nullptr,
                                                             nullptr, s);
            if (st) return st;
        }
        if ((st = exclusive_scan(counts, n, row_ptr, tiles, s))) return st;
    }
    int64_t nnz = 0;
    VCT_HIP_CHECK(hipMemcpyAsync(&nnz, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    VCT_HIP_CHECK(hipStreamSynchronize(s));
    *nnz_out = nnz;
    if (!col) return VCT_OK;
    if (col_cap < nnz) return VCT_E_CAPACITY;
    if (nnz > INT32_MAX * 8LL) return VCT_E_CAPACITY;
    if (n > 0) {
        st = (dim == 2) ? launch_neighbors<2, 16, true>(n, pos_sorted, g, R2, cell_start, nullptr, row_ptr, col, s)
                        : launch_neighbors<3, 64, true>(n, pos_sorted, g, R2, cell_start, nullptr, row_ptr, col, s);
        if (st) return st;
    }
    return VCT_OK;
}
