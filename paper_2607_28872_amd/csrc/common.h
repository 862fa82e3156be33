// Internal definitions shared by the HIP translation units of libvct.
// CDNA4 (gfx950) only: 64-lane wavefronts, 8 XCDs.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>
#include <math.h>

#include "../../include/vct.h"

namespace vct {

constexpr int kWave = 64;
constexpr int kXcds = 8;

// ------------------------------------------------------------------ errors

void set_last_error(hipError_t e);

#define VCT_HIP_CHECK(expr)                         \
    do {                                            \
        hipError_t _e = (expr);                     \
        if (_e != hipSuccess) {                     \
            ::vct::set_last_error(_e);              \
            return VCT_E_HIP;                       \
        }                                           \
    } while (0)

#define VCT_LAUNCH_CHECK() VCT_HIP_CHECK(hipGetLastError())

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------------ device checks

// A build with VCT_DEVICE_CHECKS=1 (the package's build with checks=True)
// bounds-checks the indices that kernels derive from the neighbour data: a
// failed check sets a bit of its translation unit's check word and replaces
// the index by 0, which stays inside the buffer, so the kernel still runs to
// its end; vct_device_checks reads and clears the words.  Other builds
// compile the checks out.
#ifndef VCT_DEVICE_CHECKS
#define VCT_DEVICE_CHECKS 0
#endif
enum : uint32_t {
    kChkWindow = VCT_CHECK_WINDOW,       // a window offset at or past the end of its window
    kChkCapacity = VCT_CHECK_CAPACITY,   // an index past the buffer a count is staged in
    kChkAccum = VCT_CHECK_ACCUM,         // an accumulator past the column window (push form)
};
#if VCT_DEVICE_CHECKS
[[maybe_unused]] static __device__ unsigned int g_checks;
#endif

// idx when 0 <= idx < lim; else, in a checked build, flag `bit` and return 0
template <class I, class L>
__device__ __forceinline__ I dcheck(I idx, L lim, uint32_t bit) {
#if VCT_DEVICE_CHECKS
    if (!((long long)idx >= 0 && (long long)idx < (long long)lim)) {
        atomicOr(&g_checks, bit);
        return I(0);
    }
#endif
    return idx;
}

// Host: OR this translation unit's check word into *out and clear it (after
// the device has finished the work that may set it).
#if VCT_DEVICE_CHECKS
#define VCT_CHECKS_TU(NAME)                                                                \
    int NAME(uint32_t* out) {                                                              \
        unsigned int v = 0, z = 0;                                                         \
        VCT_HIP_CHECK(hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_checks), sizeof v, 0,          \
                                          hipMemcpyDeviceToHost));                         \
        VCT_HIP_CHECK(hipMemcpyToSymbol(HIP_SYMBOL(g_checks), &z, sizeof z, 0,            \
                                        hipMemcpyHostToDevice));                           \
        *out |= v;                                                                         \
        return VCT_OK;                                                                     \
    }
#else
#define VCT_CHECKS_TU(NAME) \
    int NAME(uint32_t*) { return VCT_OK; }
#endif

// ------------------------------------------------------------------ launch timing

// While launch timing is on (vct_timing_enable), every launch is bracketed by
// two events recorded on its stream; the records are folded per kernel name by
// vct_timing_get.  When off, a launch pays one relaxed atomic load.
bool timing_on();
int timing_begin(const char* name, hipStream_t s);
void timing_end(int rec, hipStream_t s);

struct LaunchTimer {
    int rec = -1;
    hipStream_t s;
    LaunchTimer(const char* name, hipStream_t st) : s(st) {
        if (timing_on()) rec = timing_begin(name, st);
    }
    ~LaunchTimer() {
        if (rec >= 0) timing_end(rec, s);
    }
};

// A roctx range around every C-ABI entry point, named after it, so that a
// profiler run with marker tracing (rocprofv3 --marker-trace) shows the
// library's calls on the host timeline around the kernels they launch.  When
// no tool is attached the two calls return at once.
struct ApiRange {
    explicit ApiRange(const char* name) { roctxRangePushA(name); }
    ~ApiRange() { roctxRangePop(); }
    ApiRange(const ApiRange&) = delete;
    ApiRange& operator=(const ApiRange&) = delete;
};
#define VCT_API_RANGE(NAME) ::vct::ApiRange _vct_api_range(NAME)

#define VCT_LAUNCH(NAME, KERNEL, GRID, BLOCK, SHM, STREAM, ...)            \
    do {                                                                  \
        ::vct::LaunchTimer _vct_lt((NAME), (STREAM));                     \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHM, STREAM, __VA_ARGS__); \
    } while (0)

// Workspace carving: 256-byte aligned slices of a caller buffer.
struct Carver {
    char* base;
    size_t off = 0;
    size_t cap;
    Carver(void* p, size_t c) : base(static_cast<char*>(p)), cap(c) {}
    template <class T> T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += count * sizeof(T);
        return p;
    }
    bool ok() const { return off <= cap; }
};

inline size_t aligned_sum(std::initializer_list<size_t> sizes) {
    size_t off = 0;
    for (size_t s : sizes) off = ((off + 255) & ~size_t(255)) + s;
    return off + 256;
}

// ------------------------------------------------------------------ launch shape

// Work-groups are dispatched round robin over the 8 XCDs, each with its own L2.
// Remapping the dispatch index so that every XCD walks one contiguous range of
// logical tiles keeps the neighbour gathers of consecutive cell-sorted
// particles inside one L2.  The map is a bijection for any grid size.
__device__ __forceinline__ uint32_t xcd_tile(uint32_t b, uint32_t nblocks) {
    uint32_t per = nblocks / kXcds, rem = nblocks % kXcds;
    uint32_t x = b % kXcds, idx = b / kXcds;
    return x * per + (x < rem ? x : rem) + idx;
}

// Value of another lane of the same row of 16, by a DPP permutation (a VALU
// operand modifier: no LDS traffic, unlike a generic shuffle).
template <int CTRL>
__device__ __forceinline__ float dpp_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_lane(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over aligned groups of G lanes (a power of two up to the wave), the
// total in every lane of the group.  Within 16 lanes the partner lanes come
// from DPP: quad permutations (lane ^ 1, lane ^ 2), then the half-row and
// row mirrors (lane i <-> 7 - i, i <-> 15 - i), which pair every quad, then
// every half-row, with the other; wider groups use shuffles.
template <class T>
__device__ __forceinline__ T group_sum(T v, int G) {
    if (G >= 2) v += dpp_lane<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    if (G >= 4) v += dpp_lane<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    if (G >= 8) v += dpp_lane<0x141>(v);   // row_half_mirror
    if (G >= 16) v += dpp_lane<0x140>(v);  // row_mirror
    for (int m = 16; m < G; m <<= 1) v += __shfl_xor(v, m, kWave);
    return v;
}

// ------------------------------------------------------------------ background cells

struct Grid {
    double lo[3];
    double inv_cs[3];
    int64_t nc[3];
};

inline int64_t grid_setup(int dim, const double* lo, const double* hi, double R, Grid& g) {
    const double slack = R * (1.0 + 0x1p-20);
    int64_t total = 1;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = 0.0; g.inv_cs[a] = 0.0; g.nc[a] = 1;
        if (a < dim) {
            double ext = hi[a] - lo[a];
            if (!(ext > 0.0) || !isfinite(ext)) return VCT_E_ARG;
            double c = floor(ext / slack);
            int64_t nc = (c < 1.0) ? 1 : (int64_t)c;
            if (nc > (int64_t(1) << 20)) return VCT_E_ARG;
            g.lo[a] = lo[a];
            g.nc[a] = nc;
            g.inv_cs[a] = (double)nc / ext;
        }
        total *= g.nc[a];
        if (total > (int64_t(1) << 31) - 2) return VCT_E_ARG;
    }
    return total;
}

__device__ __forceinline__ int64_t cell_coord(double v, double lo, double inv, int64_t nc) {
    double t = floor((v - lo) * inv);
    if (!(t >= 0.0)) return 0;  // negative or NaN
    if (t >= (double)(nc - 1)) return nc - 1;
    return (int64_t)t;
}

__device__ __forceinline__ int64_t cell_key(int64_t c0, int64_t c1, int64_t c2, const Grid& g) {
    return (c0 * g.nc[1] + c1) * g.nc[2] + c2;
}

// ------------------------------------------------------------------ Taylor monomials

// number of unknown second derivatives and of symmetric monomials
template <int D> struct Dims;
template <> struct Dims<2> { static constexpr int m = 3, nL = 3, n3 = 4, n4 = 5, nk = 5; };
template <> struct Dims<3> { static constexpr int m = 6, nL = 6, n3 = 10, n4 = 15, nk = 9; };

// Component pairs of q (and of the symmetric correction matrix):
//   2-D (axes x, z): [xx, zz, xz];   3-D: [xx, yy, zz, xy, xz, yz]
template <int D> __host__ __device__ constexpr int pair_a(int p) {
    return D == 2 ? (p == 0 ? 0 : p == 1 ? 1 : 0)
                  : (p < 3 ? p : p == 3 ? 0 : p == 4 ? 0 : 1);
}
template <int D> __host__ __device__ constexpr int pair_b(int p) {
    return D == 2 ? (p == 0 ? 0 : 1) : (p < 3 ? p : p == 3 ? 1 : 2);
}

// position of element (a, b) of a symmetric d x d matrix stored in pairs order
template <int D> __host__ __device__ constexpr int sym_index(int a, int b) {
    return a == b ? a : (D == 2 ? 2 : ((a + b) == 1 ? 3 : (a + b) == 2 ? 4 : 5));
}

// Sorted index tuples of the 3rd- and 4th-order monomials, enumerated in
// lexicographic order of non-decreasing component tuples.
template <int D, int K> __host__ __device__ constexpr int mono_count() {
    return D == 2 ? (K == 3 ? 4 : 5) : (K == 3 ? 10 : 15);
}
// component `slot` of monomial t
template <int D, int K> __host__ __device__ constexpr int mono_comp(int t, int slot) {
    int idx = 0;
    for (int a = 0; a < D; ++a)
        for (int b = a; b < D; ++b)
            for (int c = b; c < D; ++c) {
                if (K == 3) {
                    if (idx == t) return slot == 0 ? a : slot == 1 ? b : c;
                    ++idx;
                } else {
                    for (int e = c; e < D; ++e) {
                        if (idx == t) return slot == 0 ? a : slot == 1 ? b : slot == 2 ? c : e;
                        ++idx;
                    }
                }
            }
    return -1;
}
// index of the monomial with the (unsorted) components given
template <int D> __host__ __device__ constexpr int mono3_index(int a, int b, int c) {
    int s0 = a < b ? a : b, s1 = a < b ? b : a;
    int t0 = 0, t1 = 0, t2 = 0;
    if (c < s0) { t0 = c; t1 = s0; t2 = s1; }
    else if (c < s1) { t0 = s0; t1 = c; t2 = s1; }
    else { t0 = s0; t1 = s1; t2 = c; }
    int idx = 0;
    for (int x = 0; x < D; ++x)
        for (int y = x; y < D; ++y)
            for (int z = y; z < D; ++z) {
                if (x == t0 && y == t1 && z == t2) return idx;
                ++idx;
            }
    return -1;
}
template <int D> __host__ __device__ constexpr int mono4_index(int a, int b, int c, int e) {
    int v[4] = {a, b, c, e};
    for (int i = 1; i < 4; ++i)
        for (int j = i; j > 0 && v[j - 1] > v[j]; --j) { int t = v[j]; v[j] = v[j - 1]; v[j - 1] = t; }
    int idx = 0;
    for (int x = 0; x < D; ++x)
        for (int y = x; y < D; ++y)
            for (int z = y; z < D; ++z)
                for (int w = z; w < D; ++w) {
                    if (x == v[0] && y == v[1] && z == v[2] && w == v[3]) return idx;
                    ++idx;
                }
    return -1;
}

// ------------------------------------------------------------------ kernel gradient

// Square root and reciprocal of the pair terms (kernel weights and powers of
// |r|).  FP32: the hardware instructions.  FP64: the hardware estimates are
// good to about 2^-26 only, so each gets one Newton step (the error squares to
// about an ulp), a few instructions instead of the correctly rounded library
// sequences.
template <class T> __device__ __forceinline__ T vsqrt(T x);
template <> __device__ __forceinline__ double vsqrt<double>(double x) {
    // y ~ 1/sqrt(x); y <- y (3 - x y^2) / 2; sqrt(x) = x y  (x = 0 gives 0)
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x, y * y, 1.5);
    return x > 0.0 ? x * y : 0.0;
}
template <> __device__ __forceinline__ float vsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

// 1/sqrt(x) for x > 0, the same refined estimate as vsqrt uses
__device__ __forceinline__ double vrsq(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * fma(-0.5 * x, y * y, 1.5);
}

template <class T> __device__ __forceinline__ T vrcp(T x);
template <> __device__ __forceinline__ double vrcp<double>(double x) {
    double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}
template <> __device__ __forceinline__ float vrcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }

// grad_i w(|r_ij|) = K * c~(q) * r~_ij with r~ = r/R, q = |r~|; the constant K
// (normalisation, powers of R) cancels in every corrected operator, so only
// the dimensionless shape c~ is evaluated.
//   Wendland C2, w ~ (1-q)^4 (1+4q):      c~ = (1-q)^3
//   cubic spline with l = R/2, s = 2q:     c~ = 3 - 9/4 s      (s <= 1)
//                                          c~ = 3/4 (2-s)^2/s  (1 < s < 2)
template <int KERNEL, class T>
__device__ __forceinline__ T kernel_shape(T q) {
    if (KERNEL == VCT_KERNEL_WENDLAND_C2) {
        T t = T(1) - q;
        t = t > T(0) ? t : T(0);
        return t * t * t;
    } else {
        // both branches evaluated and one selected (no divergence)
        const T s = T(2) * q;
        const T inner = T(3) - T(2.25) * s;
        T t = T(2) - s;
        t = t > T(0) ? t : T(0);
        const T outer = T(0.75) * t * t * vrcp(s);
        return s <= T(1) ? inner : outer;
    }
}



// ------------------------------------------------------------------ state layout

inline int n_out_rows(int dim, uint32_t mask) {
    int d = dim, m = dim == 2 ? 3 : 6, nc = dim == 2 ? 1 : 3;
    int n = 0;
    if (mask & VCT_OUT_GRAD) n += d;
    if (mask & VCT_OUT_LAP) n += 1;
    if (mask & VCT_OUT_CROSS) n += nc;
    if (mask & VCT_OUT_HESS) n += m;
    if (mask & VCT_OUT_PGRAD) n += d;
    if (mask & VCT_OUT_PHESS) n += m;
    if (mask & VCT_OUT_PZ) n += d + 1;
    return n;
}

inline bool mask_valid(uint32_t mask) {
    const uint32_t outs = VCT_OUT_GRAD | VCT_OUT_LAP | VCT_OUT_CROSS | VCT_OUT_HESS | VCT_OUT_PGRAD |
                          VCT_OUT_PHESS | VCT_OUT_PZ;
    return (mask & outs) != 0 && (mask & ~(outs | VCT_OPT_GRAD1)) == 0;
}

// first output row of a group within the record, or -1 if not selected
inline int group_row(int dim, uint32_t mask, uint32_t group) {
    if (!(mask & group)) return -1;
    int row = 0;
    const uint32_t order[7] = {VCT_OUT_GRAD, VCT_OUT_LAP, VCT_OUT_CROSS, VCT_OUT_HESS, VCT_OUT_PGRAD,
                               VCT_OUT_PHESS, VCT_OUT_PZ};
    for (uint32_t g : order) {
        if (g == group) return row;
        if (mask & g) row += n_out_rows(dim, g);
    }
    return -1;
}

}  // namespace vct
