// Pressure step of the projection method through the vertical coordinate
// transformation (paper Sec. 3.3, Eqs. VCT_ppe, VCT_ppe_w, VCT_predictor):
//   right-hand side  rhs_i = rho/dt div_i + gamma (rho jr_i - dens_i) / dt^2
//                    with div_i = sum_{I,K} J_IK <d v_I / d x^_K>^(1)_i (the
//                    physical divergence through the J-mapped first-order
//                    projected gradients, Eqs. div_1st and jacobi), dens_i the
//                    projected-space kernel-sum density and jr_i = Jbar_i / J_i;
//   pressure solve   c_trans . <D^ p>_i = rhs_i on ordinary rows, p_i = rhs_i on
//                    Dirichlet rows, by BiCGSTAB with the SPH(2) Laplacian of
//                    vct_apply_ops as the matrix-free operator;
//   corrector        v_i = v*_i - dt/rho J <grad^ p>^(1)_i (Eqs. gra_1st, grad_VCT).
#include <string.h>

#include "common.h"
#include "lapw.h"
#include "map_dev.h"
#include "tiles.h"

namespace vct {

int nlist_check(const vct_nlist* nl, Grid& g);

constexpr int kQLanes = 8;                    // lanes per particle
constexpr int kQThreads = kChunk * kQLanes;   // one chunk per work-group
constexpr int kQWin = 1600;                   // LDS window capacity (records)
constexpr int kQWinF = 1400;                  // the same with the fields beside the records

struct PpeArgs {
    int64_t n;
    double invR, R;
    Grid g;
    const double* pos;
    const double* vol;
    const double* state;
    int lap_row;
    const int64_t* row_ptr;
    const uint16_t* col16;
    const int64_t* cs;
    const int32_t* cstart;
    const int4* cinfo;
    const int32_t* cwin;
    const int64_t* nchunks;
    const double* f;          // [nc][n] fields (velocity components, or the pressure)
    const double* vstar;      // [dim][n] (corrector)
    const double* jr;         // [n] or NULL
    const uint8_t* dirichlet; // [n] or NULL
    const double* pbc;        // [n] or NULL
    double rho, dt, gamma;
    double* rhs;
    double* div;
    double* dens;
    double* vout;             // [dim][n] (corrector)
    double* dinv;             // [n] (Jacobi diagonal)
};

// Normalised kernel value w(q R) (unit integral): Wendland C2
// C (1 - q)^4 (1 + 4 q), C = 7 / (pi R^2) in 2-D and 21 / (2 pi R^3) in 3-D;
// cubic spline of Sec. 3.1 with l = R / 2, s = 2 q.
template <int D, int KERNEL>
__device__ __forceinline__ double kernel_value(double q, double R) {
    if (KERNEL == VCT_KERNEL_WENDLAND_C2) {
        const double C = D == 2 ? 7.0 / (M_PI * R * R) : 21.0 / (2.0 * M_PI * R * R * R);
        double t = 1.0 - q;
        t = t > 0.0 ? t : 0.0;
        const double t2 = t * t;
        return C * t2 * t2 * (1.0 + 4.0 * q);
    } else {
        const double l = 0.5 * R;
        const double ad = D == 2 ? 10.0 / (7.0 * M_PI * l * l) : 1.0 / (M_PI * l * l * l);
        const double s = 2.0 * q;
        double t = 2.0 - s;
        t = t > 0.0 ? t : 0.0;
        return s <= 1.0 ? ad * (1.0 - 1.5 * s * s + 0.75 * s * s * s) : ad * 0.25 * t * t * t;
    }
}

// One chunk per work-group, kQLanes lanes per particle: the first-order sums
// a_c = sum_j V_j c~ f_c,ij r~_ij of nc fields (and, MODE 0, the kernel sum),
// then the particle's epilogue:
//   MODE 0: right-hand side (nc = dim velocity components);
//   MODE 1: corrector (nc = 1, the pressure).
template <int D, int KERNEL, int MODE>
__global__ __launch_bounds__(kQThreads, 4) void k_ppe_first(PpeArgs A, MapParams mp) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL;
    constexpr int NC = MODE == 0 ? D : 1;
    // window records in LDS: position and volume, and the fields
    __shared__ double4 sd[kQWinF];
    __shared__ double sf[NC][kQWinF];
    __shared__ WindowT<D> w;
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *A.nchunks) return;   // uniform over the work-group
    const int64_t n = A.n;
    const int64_t p0 = A.cstart[b], p1 = A.cstart[b + 1];
    if (threadIdx.x < kWave) {
        if (A.cwin) window_load<D>(A.cwin, b, w);
        else chunk_window_wave<D>(A.g, A.cs, A.cinfo[b], w);
    }
    const int lane = threadIdx.x % kQLanes;
    const int64_t i = p0 + threadIdx.x / kQLanes;
    const bool valid = i < p1;
    const int64_t ii = valid ? i : p0;
    double xi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xi[a] = a < D ? A.pos[a * n + ii] : 0.0;
    double fi[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) fi[c] = A.f[(int64_t)c * n + ii];
    __syncthreads();
    const int W = w.off[w.nr];
    const bool in_lds = W <= kQWinF;
    if (in_lds) {
        for (int t = threadIdx.x; t < W; t += kQThreads) {
            const int64_t j = window_global<D>(w, t);
            sd[t] = make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
#pragma unroll
            for (int c = 0; c < NC; ++c) sf[c][t] = A.f[(int64_t)c * n + j];
        }
    }
    __syncthreads();
    double acc[NC][D];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int a = 0; a < D; ++a) acc[c][a] = 0.0;
    double ksum = 0.0;
    const int64_t rb = valid ? A.row_ptr[ii] : 0, re = valid ? A.row_ptr[ii + 1] : 0;
    for (int64_t e = rb + lane; e < re; e += kQLanes) {
        const int t = dcheck((int)A.col16[e], W, kChkWindow);
        double4 q;
        double fj[NC];
        if (in_lds) {
            q = sd[t];
#pragma unroll
            for (int c = 0; c < NC; ++c) fj[c] = sf[c][t];
        } else {
            const int64_t j = window_global<D>(w, t);
            q = make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
#pragma unroll
            for (int c = 0; c < NC; ++c) fj[c] = A.f[(int64_t)c * n + j];
        }
        double r[D];
        r[0] = (q.x - xi[0]) * A.invR;
        r[1] = (q.y - xi[1]) * A.invR;
        if (D == 3) r[D - 1] = (q.z - xi[2]) * A.invR;
        double q2 = r[0] * r[0];
#pragma unroll
        for (int a = 1; a < D; ++a) q2 = fma(r[a], r[a], q2);
        const double qn = vsqrt(q2);
        const double vc = q.w * kernel_shape<KERNEL>(qn);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double fij = vc * (fj[c] - fi[c]);
#pragma unroll
            for (int a = 0; a < D; ++a) acc[c][a] = fma(fij, r[a], acc[c][a]);
        }
        if (MODE == 0) ksum = fma(q.w, kernel_value<D, KERNEL>(qn, A.R), ksum);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int a = 0; a < D; ++a) acc[c][a] = group_sum(acc[c][a], kQLanes);
    if (MODE == 0) ksum = group_sum(ksum, kQLanes);
    if (!valid || lane != 0) return;
    // first-order projected gradients G_c = L~ a_c / R
    double L2[nL];
    bool ok = true;
#pragma unroll
    for (int p = 0; p < nL; ++p) {
        L2[p] = A.state[(int64_t)p * n + ii];
        ok = ok && isfinite(L2[p]);
    }
    double G[NC][3];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double g[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double t = 0.0;
#pragma unroll
            for (int bb = 0; bb < D; ++bb) t += L2[sym_index<D>(a, bb)] * acc[c][bb];
            g[a] = t * A.invR;
        }
        // 3-D component order (2-D: x^, 0, z^)
        G[c][0] = g[0];
        G[c][1] = D == 3 ? g[1] : 0.0;
        G[c][2] = g[D - 1];
    }
    // the Jacobian column of z^ at the particle: J = [[1,0,gx],[0,1,gy],[0,0,alpha]]
    const MapCoef<double> mc = map_coef_at(mp, ii, xi[0], D == 3 ? xi[1] : 0.0, xi[D - 1]);
    const double nanv = __builtin_nan("");
    if (MODE == 0) {
        // physical divergence: sum_I (J grad^ v_I)_I; component I along physical axis I
        const double gxy[2] = {mc.gx, mc.gy};
        double dv = 0.0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const int Ip = D == 3 ? c : (c == 0 ? 0 : 2);
            dv += Ip < 2 ? G[c][Ip] + gxy[Ip] * G[c][2] : mc.alpha * G[c][2];
        }
        double wself = kernel_value<D, KERNEL>(0.0, A.R);
        double ds = A.rho * fma(A.vol[ii], wself, ksum);
        if (!ok) dv = ds = nanv;
        if (A.div) A.div[ii] = dv;
        if (A.dens) A.dens[ii] = ds;
        const double jri = A.jr ? A.jr[ii] : 1.0;
        const bool dir = A.dirichlet && A.dirichlet[ii];
        A.rhs[ii] = dir ? (A.pbc ? A.pbc[ii] : 0.0)
                        : A.rho / A.dt * dv + A.gamma * (A.rho * jri - ds) / (A.dt * A.dt);
    } else {
        // physical pressure gradient J grad^ p
        const double gp[3] = {G[0][0] + mc.gx * G[0][2], G[0][1] + mc.gy * G[0][2], mc.alpha * G[0][2]};
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const int Ip = D == 3 ? c : (c == 0 ? 0 : 2);
            const double g = ok ? gp[Ip] : nanv;
            A.vout[(int64_t)c * n + ii] = A.vstar[(int64_t)c * n + ii] - A.dt / A.rho * g;
        }
    }
}

// Jacobi diagonal of the pressure system: the coefficient of p_i in row i,
// -sum_j W_ij on ordinary rows, 1 on Dirichlet rows; dinv = its inverse.
template <int D, int KERNEL>
__global__ __launch_bounds__(kQThreads, 2) void k_ppe_diag(PpeArgs A) {
    using Dm = Dims<D>;
    constexpr int nL = Dm::nL, nk = Dm::nk;
    __shared__ double4 sd[kQWin];
    __shared__ WindowT<D> w;
    const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
    if (b >= *A.nchunks) return;
    const int64_t n = A.n;
    const int64_t p0 = A.cstart[b], p1 = A.cstart[b + 1];
    if (threadIdx.x < kWave) {
        if (A.cwin) window_load<D>(A.cwin, b, w);
        else chunk_window_wave<D>(A.g, A.cs, A.cinfo[b], w);
    }
    const int lane = threadIdx.x % kQLanes;
    const int64_t i = p0 + threadIdx.x / kQLanes;
    const bool valid = i < p1;
    const int64_t ii = valid ? i : p0;
    double xi[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) xi[a] = a < D ? A.pos[a * n + ii] : 0.0;
    double L2[nL], Pl[nk];
#pragma unroll
    for (int p = 0; p < nL; ++p) L2[p] = (pair_a<D>(p) == pair_b<D>(p) ? 1.0 : 2.0) * A.state[(int64_t)p * n + ii];
#pragma unroll
    for (int c = 0; c < nk; ++c) Pl[c] = A.state[(int64_t)(nL + A.lap_row * nk + c) * n + ii];
    __syncthreads();
    const int W = w.off[w.nr];
    const bool in_lds = W <= kQWin;
    if (in_lds) {
        for (int t = threadIdx.x; t < W; t += kQThreads) {
            const int64_t j = window_global<D>(w, t);
            sd[t] = make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
        }
    }
    __syncthreads();
    double s = 0.0;
    const int64_t rb = valid ? A.row_ptr[ii] : 0, re = valid ? A.row_ptr[ii + 1] : 0;
    for (int64_t e = rb + lane; e < re; e += kQLanes) {
        const int t = dcheck((int)A.col16[e], W, kChkWindow);
        double4 q;
        if (in_lds) {
            q = sd[t];
        } else {
            const int64_t j = window_global<D>(w, t);
            q = make_double4(A.pos[j], A.pos[n + j], D == 3 ? A.pos[2 * n + j] : 0.0, A.vol[j]);
        }
        s += lap_weight<D, KERNEL>(q, xi, A.invR, L2, Pl);
    }
    s = group_sum(s, kQLanes);
    if (valid && lane == 0) {
        const bool dir = A.dirichlet && A.dirichlet[ii];
        A.dinv[ii] = dir ? 1.0 : 1.0 / (-s);
    }
}

// ------------------------------------------------------------------ BiCGSTAB

// Vector kernels run a fixed grid (kVBlocks x kVThreads, grid-stride), so each
// dot product is the same fixed-order sum on every run: per thread in index
// order, per wave and work-group in lane and wave order, then the kVBlocks
// partials in order by one work-group.  Scalars stay on the device.
constexpr int kVThreads = 256;
constexpr int kVBlocks = 1024;
constexpr int kVSlots = 3;   // partial sums per launch

// scalar slots
enum { S_RHO0, S_RHO1, S_ALPHA, S_OMEGA, S_BB, S_RR, S_DONE, S_ITERS, S_STATUS, S_RES, kNScalars };
// status values
enum { ST_RUNNING = 0, ST_CONVERGED = 1, ST_BREAKDOWN = 2, ST_MAXIT = 3 };

struct BicgVec {
    int64_t n;
    int nout, lap_row;
    const uint8_t* dirichlet;
    const double* b;
    double *x, *r, *rh, *p, *v, *s, *t, *ph, *sh, *dinv, *tmp, *part, *sc;
};

__device__ __forceinline__ void block_partials(double (&v)[kVSlots], int ns, double* part) {
    __shared__ double red[kVSlots][kVThreads / kWave];
    const int wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
    for (int k = 0; k < ns; ++k) {
        const double s = group_sum(v[k], kWave);
        if (ln == 0) red[k][wv] = s;
    }
    __syncthreads();
    if ((int)threadIdx.x < ns) {
        double s = 0.0;
        for (int w2 = 0; w2 < kVThreads / kWave; ++w2) s += red[threadIdx.x][w2];
        part[threadIdx.x * kVBlocks + blockIdx.x] = s;
    }
}

// A x on the pressure system from the operator's output tmp (the Laplacian row)
__device__ __forceinline__ double sys_row(const BicgVec& V, int64_t i, const double* xin) {
    return (V.dirichlet && V.dirichlet[i]) ? xin[i] : V.tmp[i * V.nout + V.lap_row];
}

// stage 0: r = b - A x0, r^ = r, p = v = 0; partials (r^, r), (r, r), (b, b)
__global__ __launch_bounds__(kVThreads) void k_bicg_init(BicgVec V) {
    double acc[kVSlots] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kVThreads + threadIdx.x; i < V.n; i += (int64_t)kVBlocks * kVThreads) {
        const double ri = V.b[i] - sys_row(V, i, V.x);
        V.r[i] = ri;
        V.rh[i] = ri;
        V.p[i] = 0.0;
        V.v[i] = 0.0;
        acc[0] += ri * ri;
        acc[1] += ri * ri;
        acc[2] += V.b[i] * V.b[i];
    }
    block_partials(acc, 3, V.part);
}

// sums of the partials of the last vector kernel, and the scalar updates
enum { R_INIT, R_ALPHA, R_OMEGA, R_NEXT, R_RES };
__global__ __launch_bounds__(kVBlocks) void k_bicg_reduce(double* __restrict__ part, double* __restrict__ sc, int stage,
                                                          double tol2, int maxit) {
    __shared__ double red[kVSlots][kVBlocks / kWave];
    if (stage != R_INIT && stage != R_RES && sc[S_DONE] != 0.0) return;   // uniform
    const int ns = stage == R_ALPHA ? 1 : stage == R_RES ? 1 : stage == R_INIT ? 3 : 2;
    const int wv = threadIdx.x / kWave, ln = threadIdx.x % kWave;
    for (int k = 0; k < ns; ++k) {
        const double s = group_sum(part[k * kVBlocks + threadIdx.x], kWave);
        if (ln == 0) red[k][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double d[kVSlots] = {0.0, 0.0, 0.0};
    for (int k = 0; k < ns; ++k)
        for (int w2 = 0; w2 < kVBlocks / kWave; ++w2) d[k] += red[k][w2];
    switch (stage) {
    case R_INIT:
        sc[S_RHO1] = d[0];
        sc[S_RR] = d[1];
        sc[S_BB] = d[2];
        sc[S_RHO0] = sc[S_ALPHA] = sc[S_OMEGA] = 1.0;
        sc[S_ITERS] = 0.0;
        sc[S_STATUS] = ST_RUNNING;
        sc[S_DONE] = 0.0;
        if (d[1] <= tol2 * d[2]) { sc[S_DONE] = 1.0; sc[S_STATUS] = ST_CONVERGED; }
        if (maxit <= 0 && sc[S_DONE] == 0.0) { sc[S_DONE] = 1.0; sc[S_STATUS] = ST_MAXIT; }
        break;
    case R_ALPHA:
        if (d[0] == 0.0 || !isfinite(d[0])) { sc[S_DONE] = 1.0; sc[S_STATUS] = ST_BREAKDOWN; }
        else sc[S_ALPHA] = sc[S_RHO1] / d[0];
        break;
    case R_OMEGA:   // d[0] = (t, s), d[1] = (t, t)
        if (d[1] == 0.0 || !isfinite(d[1])) { sc[S_DONE] = 1.0; sc[S_STATUS] = ST_BREAKDOWN; }
        else sc[S_OMEGA] = d[0] / d[1];
        break;
    case R_NEXT:    // d[0] = (r^, r), d[1] = (r, r)
        sc[S_RHO0] = sc[S_RHO1];
        sc[S_RHO1] = d[0];
        sc[S_RR] = d[1];
        sc[S_ITERS] += 1.0;
        if (d[1] <= tol2 * sc[S_BB]) { sc[S_DONE] = 1.0; sc[S_STATUS] = ST_CONVERGED; }
        else if (!isfinite(d[1])) { sc[S_DONE] = 1.0; sc[S_STATUS] = ST_BREAKDOWN; }
        else if (sc[S_ITERS] >= maxit) { sc[S_DONE] = 1.0; sc[S_STATUS] = ST_MAXIT; }
        break;
    case R_RES:
        sc[S_RES] = d[0];
        break;
    }
}

// p = r + beta (p - omega v), p^ = dinv p
__global__ __launch_bounds__(kVThreads) void k_bicg_p(BicgVec V) {
    if (V.sc[S_DONE] != 0.0) return;
    const double beta = (V.sc[S_RHO1] / V.sc[S_RHO0]) * (V.sc[S_ALPHA] / V.sc[S_OMEGA]);
    const double om = V.sc[S_OMEGA];
    for (int64_t i = (int64_t)blockIdx.x * kVThreads + threadIdx.x; i < V.n; i += (int64_t)kVBlocks * kVThreads) {
        const double pi = V.r[i] + beta * (V.p[i] - om * V.v[i]);
        V.p[i] = pi;
        V.ph[i] = V.dinv[i] * pi;
    }
}

// v = A p^; partial (r^, v)
__global__ __launch_bounds__(kVThreads) void k_bicg_v(BicgVec V) {
    if (V.sc[S_DONE] != 0.0) return;
    double acc[kVSlots] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kVThreads + threadIdx.x; i < V.n; i += (int64_t)kVBlocks * kVThreads) {
        const double vi = sys_row(V, i, V.ph);
        V.v[i] = vi;
        acc[0] += V.rh[i] * vi;
    }
    block_partials(acc, 1, V.part);
}

// s = r - alpha v, s^ = dinv s
__global__ __launch_bounds__(kVThreads) void k_bicg_s(BicgVec V) {
    if (V.sc[S_DONE] != 0.0) return;
    const double al = V.sc[S_ALPHA];
    for (int64_t i = (int64_t)blockIdx.x * kVThreads + threadIdx.x; i < V.n; i += (int64_t)kVBlocks * kVThreads) {
        const double si = V.r[i] - al * V.v[i];
        V.s[i] = si;
        V.sh[i] = V.dinv[i] * si;
    }
}

// t = A s^; partials (t, s), (t, t)
__global__ __launch_bounds__(kVThreads) void k_bicg_t(BicgVec V) {
    if (V.sc[S_DONE] != 0.0) return;
    double acc[kVSlots] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kVThreads + threadIdx.x; i < V.n; i += (int64_t)kVBlocks * kVThreads) {
        const double ti = sys_row(V, i, V.sh);
        V.t[i] = ti;
        acc[0] += ti * V.s[i];
        acc[1] += ti * ti;
    }
    block_partials(acc, 2, V.part);
}

// x += alpha p^ + omega s^, r = s - omega t; partials (r^, r), (r, r)
__global__ __launch_bounds__(kVThreads) void k_bicg_x(BicgVec V) {
    if (V.sc[S_DONE] != 0.0) return;
    const double al = V.sc[S_ALPHA], om = V.sc[S_OMEGA];
    double acc[kVSlots] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kVThreads + threadIdx.x; i < V.n; i += (int64_t)kVBlocks * kVThreads) {
        V.x[i] += al * V.ph[i] + om * V.sh[i];
        const double ri = V.s[i] - om * V.t[i];
        V.r[i] = ri;
        acc[0] += V.rh[i] * ri;
        acc[1] += ri * ri;
    }
    block_partials(acc, 2, V.part);
}

// true residual b - A x; partial (res, res)
__global__ __launch_bounds__(kVThreads) void k_bicg_res(BicgVec V) {
    double acc[kVSlots] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * kVThreads + threadIdx.x; i < V.n; i += (int64_t)kVBlocks * kVThreads) {
        const double ri = V.b[i] - sys_row(V, i, V.x);
        acc[0] += ri * ri;
    }
    block_partials(acc, 1, V.part);
}

static int ppe_common(const vct_nlist* nl, Grid& g, const double* pos_sorted, const double* vol_sorted, int kernel,
                      const double* state64, uint32_t out_mask, PpeArgs& a) {
    int st = nlist_check(nl, g);
    if (st) return st;
    if (!mask_valid(out_mask) || (kernel != VCT_KERNEL_WENDLAND_C2 && kernel != VCT_KERNEL_CUBIC_SPLINE))
        return VCT_E_ARG;
    const int dim = nl->dim;
    const int64_t n = nl->n;
    if (n > 0 && (!pos_sorted || !vol_sorted || !nl->col16 || !state64)) return VCT_E_ARG;
    const int64_t ncols = dim == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    memset(&a, 0, sizeof(a));
    a.n = n; a.R = nl->R; a.invR = 1.0 / nl->R; a.g = g; a.pos = pos_sorted; a.vol = vol_sorted; a.state = state64;
    a.lap_row = group_row(dim, out_mask, VCT_OUT_LAP);
    a.row_ptr = nl->row_ptr; a.col16 = nl->col16; a.cs = nl->cell_start; a.cstart = nl->chunk_start;
    a.cinfo = reinterpret_cast<const int4*>(nl->chunk_info); a.cwin = nl->chunk_win;
    a.nchunks = nl->chunk_off + ncols;
    return VCT_OK;
}

static int64_t chunk_cap(const vct_nlist* nl, const Grid& g) {
    const int64_t ncols = nl->dim == 3 ? g.nc[0] * g.nc[1] : g.nc[0];
    return ncols + nl->n / kChunk + 1;
}

template <int MODE>
static int launch_first(int dim, int kernel, const PpeArgs& a, const MapParams& mp, int64_t cap, hipStream_t s) {
    const char* name = MODE == 0 ? "k_ppe_first (rhs)" : "k_ppe_first (correct)";
#define VCT_PPE_FIRST(D, K) VCT_LAUNCH(name, (k_ppe_first<D, K, MODE>), dim3((unsigned)cap), dim3(kQThreads), 0, s, a, mp)
    if (dim == 2) {
        if (kernel == VCT_KERNEL_WENDLAND_C2) VCT_PPE_FIRST(2, VCT_KERNEL_WENDLAND_C2);
        else VCT_PPE_FIRST(2, VCT_KERNEL_CUBIC_SPLINE);
    } else {
        if (kernel == VCT_KERNEL_WENDLAND_C2) VCT_PPE_FIRST(3, VCT_KERNEL_WENDLAND_C2);
        else VCT_PPE_FIRST(3, VCT_KERNEL_CUBIC_SPLINE);
    }
#undef VCT_PPE_FIRST
    VCT_LAUNCH_CHECK();
    return VCT_OK;
}

VCT_CHECKS_TU(checks_ppe)

}  // namespace vct

using namespace vct;

extern "C" int vct_ppe_rhs(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                           const double* state64, uint32_t out_mask, const vct_map* map, const double* vstar,
                           double rho, double dt, double gamma, const double* jr, const uint8_t* dirichlet,
                           const double* pbc, double* rhs, double* div, double* dens, void* stream) {
    VCT_API_RANGE("vct_ppe_rhs");
    Grid g;
    PpeArgs a;
    int st = ppe_common(nl, g, pos_sorted, vol_sorted, kernel, state64, out_mask, a);
    if (st) return st;
    if (!map || !(dt > 0.0) || !isfinite(rho) || !isfinite(gamma)) return VCT_E_ARG;
    MapParams mp;
    st = map_params_from(map, nl->dim, nl->n, mp);
    if (st) return st;
    if (nl->n == 0) return VCT_OK;
    if (!vstar || !rhs) return VCT_E_ARG;
    a.f = vstar; a.jr = jr; a.dirichlet = dirichlet; a.pbc = pbc; a.rho = rho; a.dt = dt; a.gamma = gamma;
    a.rhs = rhs; a.div = div; a.dens = dens;
    return launch_first<0>(nl->dim, kernel, a, mp, chunk_cap(nl, g), as_stream(stream));
}

extern "C" int vct_ppe_correct(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                               const double* state64, uint32_t out_mask, const vct_map* map, const double* p,
                               const double* vstar, double rho, double dt, double* vout, void* stream) {
    VCT_API_RANGE("vct_ppe_correct");
    Grid g;
    PpeArgs a;
    int st = ppe_common(nl, g, pos_sorted, vol_sorted, kernel, state64, out_mask, a);
    if (st) return st;
    if (!map || !isfinite(dt) || !(rho != 0.0) || !isfinite(rho)) return VCT_E_ARG;
    MapParams mp;
    st = map_params_from(map, nl->dim, nl->n, mp);
    if (st) return st;
    if (nl->n == 0) return VCT_OK;
    if (!p || !vstar || !vout) return VCT_E_ARG;
    a.f = p; a.vstar = vstar; a.vout = vout; a.rho = rho; a.dt = dt;
    return launch_first<1>(nl->dim, kernel, a, mp, chunk_cap(nl, g), as_stream(stream));
}

extern "C" size_t vct_ppe_workspace_size(int dim, int64_t n, uint32_t out_mask) {
    if ((dim != 2 && dim != 3) || n < 0 || !mask_valid(out_mask)) return 0;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    return aligned_sum({nn * 10 * sizeof(double), nn * (size_t)n_out_rows(dim, out_mask) * sizeof(double),
                        (size_t)kVSlots * kVBlocks * sizeof(double), (size_t)kNScalars * sizeof(double)});
}

extern "C" int vct_ppe_solve(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                             const double* state64, uint32_t out_mask, const uint8_t* dirichlet, const double* rhs,
                             double* p, double tol, int max_iter, int* iters, double* relres, void* ws,
                             size_t ws_bytes, void* stream) {
    VCT_API_RANGE("vct_ppe_solve");
    Grid g;
    PpeArgs a;
    int st = ppe_common(nl, g, pos_sorted, vol_sorted, kernel, state64, out_mask, a);
    if (st) return st;
    if (!(out_mask & VCT_OUT_LAP) || !(tol >= 0.0) || max_iter < 0) return VCT_E_ARG;
    const int dim = nl->dim;
    const int64_t n = nl->n;
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    if (n == 0) return VCT_OK;
    if (!rhs || !p) return VCT_E_ARG;
    if (!ws || ws_bytes < vct_ppe_workspace_size(dim, n, out_mask)) return VCT_E_WORKSPACE;
    hipStream_t s = as_stream(stream);
    const int nout = n_out_rows(dim, out_mask);
    Carver cv(ws, ws_bytes);
    BicgVec V;
    V.n = n; V.nout = nout; V.lap_row = a.lap_row; V.dirichlet = dirichlet; V.b = rhs; V.x = p;
    double* vecs = cv.take<double>((size_t)n * 10);
    V.r = vecs; V.rh = vecs + n; V.p = vecs + 2 * n; V.v = vecs + 3 * n; V.s = vecs + 4 * n; V.t = vecs + 5 * n;
    V.ph = vecs + 6 * n; V.sh = vecs + 7 * n; V.dinv = vecs + 8 * n;
    V.tmp = cv.take<double>((size_t)n * nout);
    V.part = cv.take<double>((size_t)kVSlots * kVBlocks);
    V.sc = cv.take<double>(kNScalars);
    const int64_t cap = chunk_cap(nl, g);
    a.dirichlet = dirichlet; a.dinv = V.dinv;
    if (dim == 2) {
        if (kernel == VCT_KERNEL_WENDLAND_C2) VCT_LAUNCH("k_ppe_diag", (k_ppe_diag<2, VCT_KERNEL_WENDLAND_C2>), dim3((unsigned)cap), dim3(kQThreads), 0, s, a);
        else VCT_LAUNCH("k_ppe_diag", (k_ppe_diag<2, VCT_KERNEL_CUBIC_SPLINE>), dim3((unsigned)cap), dim3(kQThreads), 0, s, a);
    } else {
        if (kernel == VCT_KERNEL_WENDLAND_C2) VCT_LAUNCH("k_ppe_diag", (k_ppe_diag<3, VCT_KERNEL_WENDLAND_C2>), dim3((unsigned)cap), dim3(kQThreads), 0, s, a);
        else VCT_LAUNCH("k_ppe_diag", (k_ppe_diag<3, VCT_KERNEL_CUBIC_SPLINE>), dim3((unsigned)cap), dim3(kQThreads), 0, s, a);
    }
    VCT_LAUNCH_CHECK();
    const double tol2 = tol * tol;
    auto matvec = [&](const double* xin) {
        return vct_apply_ops(nl, 1, xin, pos_sorted, vol_sorted, kernel, state64, out_mask, VCT_FP64, V.tmp, stream);
    };
    const dim3 vg(kVBlocks), vb(kVThreads);
    if ((st = matvec(V.x)) < 0) return st;
    VCT_LAUNCH("k_bicg_init", k_bicg_init, vg, vb, 0, s, V);
    VCT_LAUNCH_CHECK();
    VCT_LAUNCH("k_bicg_reduce", k_bicg_reduce, dim3(1), dim3(kVBlocks), 0, s, V.part, V.sc, (int)R_INIT, tol2, max_iter);
    VCT_LAUNCH_CHECK();
    // iterations in batches; the host reads the scalars after each batch
    constexpr int kBatch = 8;
    double hs[kNScalars];
    int done_iters = 0;
    for (;;) {
        VCT_HIP_CHECK(hipMemcpyAsync(hs, V.sc, sizeof(hs), hipMemcpyDeviceToHost, s));
        VCT_HIP_CHECK(hipStreamSynchronize(s));
        if (hs[S_DONE] != 0.0 || done_iters >= max_iter) break;
        for (int k = 0; k < kBatch && done_iters < max_iter; ++k, ++done_iters) {
            VCT_LAUNCH("k_bicg_p", k_bicg_p, vg, vb, 0, s, V);
            VCT_LAUNCH_CHECK();
            if ((st = matvec(V.ph)) < 0) return st;
            VCT_LAUNCH("k_bicg_v", k_bicg_v, vg, vb, 0, s, V);
            VCT_LAUNCH_CHECK();
            VCT_LAUNCH("k_bicg_reduce", k_bicg_reduce, dim3(1), dim3(kVBlocks), 0, s, V.part, V.sc, (int)R_ALPHA, tol2, max_iter);
            VCT_LAUNCH_CHECK();
            VCT_LAUNCH("k_bicg_s", k_bicg_s, vg, vb, 0, s, V);
            VCT_LAUNCH_CHECK();
            if ((st = matvec(V.sh)) < 0) return st;
            VCT_LAUNCH("k_bicg_t", k_bicg_t, vg, vb, 0, s, V);
            VCT_LAUNCH_CHECK();
            VCT_LAUNCH("k_bicg_reduce", k_bicg_reduce, dim3(1), dim3(kVBlocks), 0, s, V.part, V.sc, (int)R_OMEGA, tol2, max_iter);
            VCT_LAUNCH_CHECK();
            VCT_LAUNCH("k_bicg_x", k_bicg_x, vg, vb, 0, s, V);
            VCT_LAUNCH_CHECK();
            VCT_LAUNCH("k_bicg_reduce", k_bicg_reduce, dim3(1), dim3(kVBlocks), 0, s, V.part, V.sc, (int)R_NEXT, tol2, max_iter);
            VCT_LAUNCH_CHECK();
        }
    }
    // the true residual of the result
    if ((st = matvec(V.x)) < 0) return st;
    VCT_LAUNCH("k_bicg_res", k_bicg_res, vg, vb, 0, s, V);
    VCT_LAUNCH_CHECK();
    VCT_LAUNCH("k_bicg_reduce", k_bicg_reduce, dim3(1), dim3(kVBlocks), 0, s, V.part, V.sc, (int)R_RES, tol2, max_iter);
    VCT_LAUNCH_CHECK();
    VCT_HIP_CHECK(hipMemcpyAsync(hs, V.sc, sizeof(hs), hipMemcpyDeviceToHost, s));
    VCT_HIP_CHECK(hipStreamSynchronize(s));
    if (iters) *iters = (int)hs[S_ITERS];
    if (relres) *relres = hs[S_BB] > 0.0 ? sqrt(hs[S_RES] / hs[S_BB]) : sqrt(hs[S_RES]);
    return hs[S_STATUS] == ST_CONVERGED ? VCT_OK : VCT_W_NOCONV;
}
