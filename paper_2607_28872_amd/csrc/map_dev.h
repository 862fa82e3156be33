// Vertical coordinate transformation on the device: bottom elevation terms,
// alpha/beta for the mapping kinds, and the coefficients that carry projected
// derivatives to physical ones (paper Sec. 2.1, Eqs. VCT, jacobi, grad_VCT,
// lap_VCT; Sec. 2.2 for alpha and beta).
//
// The same template serves plain FP64 and a forward-mode dual number whose
// tangents are the derivatives with respect to the six bottom-elevation
// quantities (h, h_x, h_y, h_xx, h_xy, h_yy); the adjoint uses the latter for
// the sensitivity to bathymetry coefficients.
#pragma once

#include "common.h"

namespace vct {

constexpr int kMapFn = 6;   // distinct factors per axis in the separable table
constexpr int kMapFq = 4;   // distinct frequencies per axis in the separable table

struct MapParams {
    int32_t kind;
    int32_t nterms;
    int32_t dim;
    int32_t limiter;          // sigma: smooth depth limiter on
    double Hhat, H, dmin, eps;
    double coef[VCT_MAX_TERMS];
    int32_t bx[VCT_MAX_TERMS], by[VCT_MAX_TERMS];
    double fx[VCT_MAX_TERMS], fy[VCT_MAX_TERMS];
    // The same bottom as h = sum_ab cm[a][b] X_a(x) Y_b(y) over the distinct
    // factors of each axis (kind and frequency slot), filled by the host when
    // the terms have at most kMapFn factors and kMapFq frequencies per axis
    // (sep = 1): each frequency's sine and cosine are then evaluated once per
    // particle instead of once per term.
    int32_t sep;
    int32_t nfx, nfy, nqx, nqy;
    int32_t fx_kind[kMapFn], fx_q[kMapFn], fy_kind[kMapFn], fy_q[kMapFn];
    double qx[kMapFq], qy[kMapFq];
    double cm[kMapFn][kMapFn];
    int32_t term_a[VCT_MAX_TERMS], term_b[VCT_MAX_TERMS];   // factors (X_a, Y_b) of every term
    // VCT_MAP_PER_PARTICLE: alpha, beta and their derivatives of every point,
    // [12][pp_n] (order of vct_map.coef)
    const double* pp;
    int64_t pp_n;
};

// host, returns status; n = the number of points of the call (checked
// against the per-particle coefficient count)
int map_params_from(const vct_map* m, int dim, int64_t n, MapParams& p);

// B(s), B'(s), B''(s) of one separable factor
__device__ __forceinline__ void basis3(int kind, double f, double s, double b[3]) {
    if (kind == VCT_BASIS_ONE) { b[0] = 1.0; b[1] = 0.0; b[2] = 0.0; return; }
    if (kind == VCT_BASIS_LIN) { b[0] = s; b[1] = 1.0; b[2] = 0.0; return; }
    double sn, cs;
    sincospi(2.0 * f * s, &sn, &cs);
    const double w = 2.0 * M_PI * f;
    if (kind == VCT_BASIS_COS) { b[0] = cs; b[1] = -w * sn; b[2] = -w * w * cs; }
    else { b[0] = sn; b[1] = w * cs; b[2] = -w * w * sn; }
}

// the six products [B B, B' B, B B', B'' B, B' B', B B''] of term t at (x, y)
__device__ __forceinline__ void term_derivs(const MapParams& mp, int t, double x, double y, double o[6]) {
    double bx[3], by[3];
    basis3(mp.bx[t], mp.fx[t], x, bx);
    basis3(mp.by[t], mp.fy[t], y, by);
    if (mp.dim == 2) { by[1] = 0.0; by[2] = 0.0; }
    o[0] = bx[0] * by[0];
    o[1] = bx[1] * by[0];
    o[2] = bx[0] * by[1];
    o[3] = bx[2] * by[0];
    o[4] = bx[1] * by[1];
    o[5] = bx[0] * by[2];
}

// F(s), F'(s), F''(s) of factor a of the separable table along one axis;
// kind and slot are uniform, so every choice is a select
__device__ __forceinline__ void sep_factor_values(int a, int nf, int kind, int q, const double (&freq)[kMapFq],
                                                  const double (&sn)[kMapFq], const double (&cs)[kMapFq],
                                                  double s, double& F0, double& F1, double& F2) {
    double vs = sn[0], vc = cs[0], f = freq[0];
#pragma unroll
    for (int j = 1; j < kMapFq; ++j) {
        vs = q == j ? sn[j] : vs;
        vc = q == j ? cs[j] : vc;
        f = q == j ? freq[j] : f;
    }
    const double w = 2.0 * M_PI * f;
    const bool on = a < nf;
    const bool c = kind == VCT_BASIS_COS, sk = kind == VCT_BASIS_SIN;
    const double t0 = c ? vc : vs, t1 = c ? -w * vs : w * vc;
    F0 = !on ? 0.0 : kind == VCT_BASIS_ONE ? 1.0 : kind == VCT_BASIS_LIN ? s : (c || sk) ? t0 : 0.0;
    F1 = !on ? 0.0 : kind == VCT_BASIS_LIN ? 1.0 : (c || sk) ? t1 : 0.0;
    F2 = !on ? 0.0 : (c || sk) ? -w * w * t0 : 0.0;
}

// Every factor of the separable table at (x, y): X*[a] = X_a, X_a', X_a''
// and the same for Y (zero y-derivatives in 2-D).
struct SepFactors {
    double X0[kMapFn], X1[kMapFn], X2[kMapFn], Y0[kMapFn], Y1[kMapFn], Y2[kMapFn];
};
__device__ __forceinline__ void sep_table(const MapParams& mp, double x, double y, SepFactors& F) {
    double sx[kMapFq], cx[kMapFq], sy[kMapFq], cy[kMapFq];
#pragma unroll
    for (int q = 0; q < kMapFq; ++q) {
        sx[q] = sy[q] = 0.0;
        cx[q] = cy[q] = 1.0;
        double sv, cv;
        if (q < mp.nqx) {
            sincospi(2.0 * mp.qx[q] * x, &sv, &cv);
            sx[q] = sv;
            cx[q] = cv;
        }
        if (q < mp.nqy) {
            sincospi(2.0 * mp.qy[q] * y, &sv, &cv);
            sy[q] = sv;
            cy[q] = cv;
        }
    }
    double qx[kMapFq], qy[kMapFq];
#pragma unroll
    for (int q = 0; q < kMapFq; ++q) {
        qx[q] = mp.qx[q];
        qy[q] = mp.qy[q];
    }
#pragma unroll
    for (int a = 0; a < kMapFn; ++a) {
        sep_factor_values(a, mp.nfx, mp.fx_kind[a], mp.fx_q[a], qx, sx, cx, x, F.X0[a], F.X1[a], F.X2[a]);
        sep_factor_values(a, mp.nfy, mp.fy_kind[a], mp.fy_q[a], qy, sy, cy, y, F.Y0[a], F.Y1[a], F.Y2[a]);
        if (mp.dim == 2) F.Y1[a] = F.Y2[a] = 0.0;
    }
}

// h, h_x, h_y, h_xx, h_xy, h_yy from the separable table's factors
__device__ __forceinline__ void bottom6_sep(const MapParams& mp, const SepFactors& F, double h[6]) {
    for (int k = 0; k < 6; ++k) h[k] = 0.0;
#pragma unroll
    for (int a = 0; a < kMapFn; ++a) {
        double u0 = 0.0, u1 = 0.0, u2 = 0.0;   // sum_b cm[a][b] (Y_b, Y_b', Y_b'')
#pragma unroll
        for (int b = 0; b < kMapFn; ++b) {
            u0 += mp.cm[a][b] * F.Y0[b];
            u1 += mp.cm[a][b] * F.Y1[b];
            u2 += mp.cm[a][b] * F.Y2[b];
        }
        h[0] += F.X0[a] * u0;
        h[1] += F.X1[a] * u0;
        h[2] += F.X0[a] * u1;
        h[3] += F.X2[a] * u0;
        h[4] += F.X1[a] * u1;
        h[5] += F.X0[a] * u2;
    }
}

// h, h_x, h_y, h_xx, h_xy, h_yy at (x, y)
__device__ __forceinline__ void bottom6(const MapParams& mp, double x, double y, double h[6]) {
    for (int k = 0; k < 6; ++k) h[k] = 0.0;
    if (mp.sep) {
        SepFactors F;
        sep_table(mp, x, y, F);
#pragma unroll
        for (int a = 0; a < kMapFn; ++a) {
            double u0 = 0.0, u1 = 0.0, u2 = 0.0;   // sum_b cm[a][b] (Y_b, Y_b', Y_b'')
#pragma unroll
            for (int b = 0; b < kMapFn; ++b) {
                u0 += mp.cm[a][b] * F.Y0[b];
                u1 += mp.cm[a][b] * F.Y1[b];
                u2 += mp.cm[a][b] * F.Y2[b];
            }
            h[0] += F.X0[a] * u0;
            h[1] += F.X1[a] * u0;
            h[2] += F.X0[a] * u1;
            h[3] += F.X2[a] * u0;
            h[4] += F.X1[a] * u1;
            h[5] += F.X0[a] * u2;
        }
        return;
    }
    for (int t = 0; t < mp.nterms; ++t) {
        double o[6];
        term_derivs(mp, t, x, y, o);
        for (int k = 0; k < 6; ++k) h[k] += mp.coef[t] * o[k];
    }
}

// ------------------------------------------------------------------ dual numbers

struct Dual6 {
    double v;
    double d[6];
    __device__ Dual6() {}
    __device__ Dual6(double c) : v(c) { for (int k = 0; k < 6; ++k) d[k] = 0.0; }
};
__device__ __forceinline__ Dual6 operator+(const Dual6& a, const Dual6& b) {
    Dual6 r; r.v = a.v + b.v; for (int k = 0; k < 6; ++k) r.d[k] = a.d[k] + b.d[k]; return r;
}
__device__ __forceinline__ Dual6 operator-(const Dual6& a, const Dual6& b) {
    Dual6 r; r.v = a.v - b.v; for (int k = 0; k < 6; ++k) r.d[k] = a.d[k] - b.d[k]; return r;
}
__device__ __forceinline__ Dual6 operator-(const Dual6& a) {
    Dual6 r; r.v = -a.v; for (int k = 0; k < 6; ++k) r.d[k] = -a.d[k]; return r;
}
__device__ __forceinline__ Dual6 operator*(const Dual6& a, const Dual6& b) {
    Dual6 r; r.v = a.v * b.v; for (int k = 0; k < 6; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r;
}
__device__ __forceinline__ Dual6 operator/(const Dual6& a, const Dual6& b) {
    Dual6 r; r.v = a.v / b.v;
    double ib = 1.0 / b.v;
    for (int k = 0; k < 6; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
    return r;
}
__device__ __forceinline__ Dual6 dsqrt(const Dual6& a) {
    Dual6 r; r.v = sqrt(a.v);
    double h = 0.5 / r.v;
    for (int k = 0; k < 6; ++k) r.d[k] = a.d[k] * h;
    return r;
}
__device__ __forceinline__ double dsqrt(double a) { return sqrt(a); }
__device__ __forceinline__ double value(double a) { return a; }
__device__ __forceinline__ double value(const Dual6& a) { return a.v; }

// ------------------------------------------------------------------ mapping coefficients

// Coefficients of the physical derivatives at one particle:
//   gx = dz^/dx, gy = dz^/dy, alpha = dz^/dz (Jacobian column of z^, Eq. jacobi)
//   c0, c3, c4, c5: the non-constant entries of c_trans (Eq. lap_VCT)
//   second derivatives of z^ with respect to (x, y, z): zxx, zyy, zxy, zxz, zyz (zzz = 0)
template <class T> struct MapCoef {
    T alpha, gx, gy, c0, c3, c4, c5, zxx, zyy, zxy, zxz, zyz;
    T beta, axx, ayy;   // beta, d2 alpha / dx2, d2 alpha / dy2
};

template <class T>
__device__ __forceinline__ MapCoef<T> map_coef_ab(T a, T ax, T ay, T axx, T axy, T ayy, T bet, T bx, T by, T bxx,
                                                  T bxy, T byy, double zh);

// From h (and derivatives) and the projected height zh; z + beta = zh / alpha.
template <class T>
__device__ __forceinline__ MapCoef<T> map_coef(const MapParams& mp, const T h[6], double zh) {
    T a(1.0), ax(0.0), ay(0.0), axx(0.0), axy(0.0), ayy(0.0);
    T bet(0.0), bx(0.0), by(0.0), bxx(0.0), bxy(0.0), byy(0.0);
    if (mp.kind == VCT_MAP_E || mp.kind == VCT_MAP_BFE) a = T(mp.Hhat / mp.H);
    if (mp.kind == VCT_MAP_BF || mp.kind == VCT_MAP_BFE) {
        bet = -h[0]; bx = -h[1]; by = -h[2]; bxx = -h[3]; bxy = -h[4]; byy = -h[5];
    }
    if (mp.kind == VCT_MAP_SIGMA) {
        // depth D = H - h, smoothly limited from below: E = smax(D, dmin; eps)
        T D = T(mp.H) - h[0];
        T Dx = -h[1], Dy = -h[2], Dxx = -h[3], Dxy = -h[4], Dyy = -h[5];
        T E = D, s1(1.0), s2(0.0);
        if (mp.limiter) {
            T dd = D - T(mp.dmin);
            T S = dsqrt(dd * dd + T(mp.eps * mp.eps));
            E = T(0.5) * (D + T(mp.dmin) + S);
            s1 = T(0.5) * (T(1.0) + dd / S);
            s2 = T(0.5 * mp.eps * mp.eps) / (S * S * S);
        }
        T Ex = s1 * Dx, Ey = s1 * Dy;
        T Exx = s2 * Dx * Dx + s1 * Dxx;
        T Exy = s2 * Dx * Dy + s1 * Dxy;
        T Eyy = s2 * Dy * Dy + s1 * Dyy;
        T iE = T(1.0) / E;
        T Hh(mp.Hhat);
        a = Hh * iE;
        ax = -a * Ex * iE;
        ay = -a * Ey * iE;
        axx = a * iE * (T(2.0) * Ex * Ex * iE - Exx);
        axy = a * iE * (T(2.0) * Ex * Ey * iE - Exy);
        ayy = a * iE * (T(2.0) * Ey * Ey * iE - Eyy);
        bet = E - T(mp.H);
        bx = Ex; by = Ey; bxx = Exx; bxy = Exy; byy = Eyy;
    }
    return map_coef_ab<T>(a, ax, ay, axx, axy, ayy, bet, bx, by, bxx, bxy, byy, zh);
}

// The coefficients from alpha, beta and their derivatives at the point
// (Eqs. jacobi, lap_VCT and the second derivatives of z^).
template <class T>
__device__ __forceinline__ MapCoef<T> map_coef_ab(T a, T ax, T ay, T axx, T axy, T ayy, T bet, T bx, T by, T bxx,
                                                  T bxy, T byy, double zh) {
    T zb = T(zh) / a;  // z + beta
    MapCoef<T> c;
    c.alpha = a;
    c.beta = bet;
    c.axx = axx;
    c.ayy = ayy;
    c.gx = ax * zb + a * bx;
    c.gy = ay * zb + a * by;
    c.zxx = axx * zb + T(2.0) * ax * bx + a * bxx;
    c.zyy = ayy * zb + T(2.0) * ay * by + a * byy;
    c.zxy = axy * zb + ax * by + ay * bx + a * bxy;
    c.zxz = ax;
    c.zyz = ay;
    c.c0 = c.zxx + c.zyy;                         // Laplacian of z^
    c.c3 = a * a + c.gx * c.gx + c.gy * c.gy;
    c.c4 = T(2.0) * c.gx;
    c.c5 = T(2.0) * c.gy;
    return c;
}

// The coefficients at point i of a call, at (x, y, zh): from the bottom
// terms, or read from the per-particle table (2-D: the y derivatives are 0).
__device__ __forceinline__ MapCoef<double> map_coef_at(const MapParams& mp, int64_t i, double x, double y, double zh) {
    if (mp.kind == VCT_MAP_PER_PARTICLE) {
        const double* c = mp.pp;
        const int64_t n = mp.pp_n;
        const bool d3 = mp.dim == 3;
        return map_coef_ab<double>(c[i], c[n + i], d3 ? c[2 * n + i] : 0.0, c[3 * n + i], d3 ? c[4 * n + i] : 0.0,
                                   d3 ? c[5 * n + i] : 0.0, c[6 * n + i], c[7 * n + i], d3 ? c[8 * n + i] : 0.0,
                                   c[9 * n + i], d3 ? c[10 * n + i] : 0.0, d3 ? c[11 * n + i] : 0.0, zh);
    }
    double h[6];
    bottom6(mp, x, y, h);
    return map_coef<double>(mp, h, zh);
}

// Physical (and projected) outputs from a projected gradient pg and projected
// second derivatives ph (pairs order), in the row order of the output mask.
// Linear in (pg, ph): applied to one column of the solved system it yields
// that column of P.  Eq. grad_VCT, Eq. lap_VCT, and the chain rule
// Hess = J H^ J^T + dz^phi (d2 z^) for the cross and full Hessian rows.
template <int D, class Put>
__device__ __forceinline__ int emit_rows(uint32_t mask, const MapCoef<double>& c, const double* pg,
                                         const double* ph, Put&& out) {
    int o = 0;
    if (D == 3) {
        const double gz = pg[2];
        const double Hxx = ph[0], Hyy = ph[1], Hzz = ph[2], Hxy = ph[3], Hxz = ph[4], Hyz = ph[5];
        const double xy = Hxy + c.gy * Hxz + c.gx * Hyz + c.gx * c.gy * Hzz + c.zxy * gz;
        const double xz = c.alpha * (Hxz + c.gx * Hzz) + c.zxz * gz;
        const double yz = c.alpha * (Hyz + c.gy * Hzz) + c.zyz * gz;
        if (mask & VCT_OUT_GRAD) {
            out(o++, pg[0] + c.gx * gz);
            out(o++, pg[1] + c.gy * gz);
            out(o++, c.alpha * gz);
        }
        if (mask & VCT_OUT_LAP) out(o++, c.c0 * gz + Hxx + Hyy + c.c3 * Hzz + c.c4 * Hxz + c.c5 * Hyz);
        if (mask & VCT_OUT_CROSS) { out(o++, xy); out(o++, xz); out(o++, yz); }
        if (mask & VCT_OUT_HESS) {
            out(o++, Hxx + 2.0 * c.gx * Hxz + c.gx * c.gx * Hzz + c.zxx * gz);
            out(o++, Hyy + 2.0 * c.gy * Hyz + c.gy * c.gy * Hzz + c.zyy * gz);
            out(o++, c.alpha * c.alpha * Hzz);
            out(o++, xy); out(o++, xz); out(o++, yz);
        }
        if (mask & VCT_OUT_PGRAD) { out(o++, pg[0]); out(o++, pg[1]); out(o++, pg[2]); }
        if (mask & VCT_OUT_PHESS) for (int p = 0; p < 6; ++p) out(o++, ph[p]);
        if (mask & VCT_OUT_PZ) { out(o++, gz); out(o++, Hzz); out(o++, Hxz); out(o++, Hyz); }
    } else {
        const double gz = pg[1];
        const double Hxx = ph[0], Hzz = ph[1], Hxz = ph[2];
        const double xz = c.alpha * (Hxz + c.gx * Hzz) + c.zxz * gz;
        if (mask & VCT_OUT_GRAD) { out(o++, pg[0] + c.gx * gz); out(o++, c.alpha * gz); }
        if (mask & VCT_OUT_LAP) out(o++, c.c0 * gz + Hxx + c.c3 * Hzz + c.c4 * Hxz);
        if (mask & VCT_OUT_CROSS) out(o++, xz);
        if (mask & VCT_OUT_HESS) {
            out(o++, Hxx + 2.0 * c.gx * Hxz + c.gx * c.gx * Hzz + c.zxx * gz);
            out(o++, c.alpha * c.alpha * Hzz);
            out(o++, xz);
        }
        if (mask & VCT_OUT_PGRAD) { out(o++, pg[0]); out(o++, pg[1]); }
        if (mask & VCT_OUT_PHESS) for (int p = 0; p < 3; ++p) out(o++, ph[p]);
        if (mask & VCT_OUT_PZ) { out(o++, gz); out(o++, Hzz); out(o++, Hxz); }
    }
    return o;
}

}  // namespace vct
