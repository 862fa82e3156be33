/* Oracle for the VCT-SPH(2) derivative operators: plain, slow, FP64 C.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no source, header, table or helper with the GPU
 * library: every formula is written out again here from the paper, in the
 * paper's own order and notation.
 *
 * What it computes, per particle i (paper Sec. 3.1):
 *   S_i        = { j != i : |r_ij| < r_e }                       (Eq. SPH_neighbor_set)
 *   L_i        = [ sum_j V_j grad w_ij (x) r_ij ]^-1              (Eq. gra_1st)
 *   g1_i       = sum_j V_j phi_ij L_i grad w_ij                   (Eq. gra_1st)
 *   F_ij       = r_ij . (L_i grad w_ij) / |r_ij|^4                (Eq. sec_SPH2)
 *   p_ij       = q_ij - (sum_k V_k q_ik (L_i grad w_ik)^T) r_ij  (Eq. sec_SPH2, see below)
 *   M_i        = sum_j V_j F_ij q_ij p_ij^T
 *   D_i        = 2 M_i^-1 sum_j V_j F_ij q_ij (phi_ij - r_ij . g1_i)
 *   grad2_i    = g1_i - 1/2 Q_i^T D_i,  Q_i = sum_k V_k q_ik (L_i grad w_ik)^T
 * then the physical derivatives through the vertical coordinate transformation
 * (paper Sec. 2.1): grad = J grad^ (Eq. grad_VCT), lap = c_trans . D^ (Eq. lap_VCT),
 * and the full physical Hessian by the chain rule J H^ J^T + phi_z^ (d2 z^).
 *
 * Readings where the paper is silent or garbled:
 *  - p_ij is printed as a scalar minus a vector; it is read as each component
 *    q_ij^m minus r_ij . sum_k V_k q_ik^m L_i grad w_ik (the only reading that
 *    reproduces quadratic fields exactly).
 *  - SPH(2) is printed for 2-D (x, y) only.  2-D sets here use the vertical
 *    plane (x, z) with q = [x^2, z^2, xz]; 3-D uses q = [x^2, y^2, z^2, xy, xz, yz]
 *    and D = [xx, yy, zz, 2xy, 2xz, 2yz].
 *  - grad w_ij is the gradient with respect to r_i of w(|r_j - r_i|); its sign
 *    and normalisation cancel in every corrected operator.
 *  - the particle itself is excluded from S_i (F_ii would be 0/0).
 *  - the neighbour test evaluates d2 = dx*dx + dy*dy (+ dz*dz) left to right in
 *    FP64 without fused multiply-add and compares d2 < R*R (strict, as printed).
 *  - the gradient reported is grad2 (second order) unless first order is asked.
 *  - the physical cross derivatives are not printed; they come from the chain
 *    rule above.
 *  - a particle with fewer than d + m neighbours, a singular A_i or M_i, a
 *    duplicate position, a non-finite input, or a mapping whose alpha is not
 *    positive and finite there (Sec. 2.1 needs alpha > 0) gets NaN outputs
 *    and a flag.
 */
#include <complex.h>
#undef I            /* loop indices below use I; the imaginary unit is _Complex_I */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "orc.h"

/* ------------------------------------------------------------------ basis */

/* One separable bathymetry factor B(s) and its first two derivatives. */
static void orc_basis(int kind, double f, double s, double b[3])
{
    const double w = 2.0 * M_PI * f;
    switch (kind) {
    case ORC_B_ONE: b[0] = 1.0; b[1] = 0.0; b[2] = 0.0; break;
    case ORC_B_LIN: b[0] = s;   b[1] = 1.0; b[2] = 0.0; break;
    case ORC_B_COS: b[0] = cos(w * s); b[1] = -w * sin(w * s); b[2] = -w * w * cos(w * s); break;
    case ORC_B_SIN: b[0] = sin(w * s); b[1] = w * cos(w * s);  b[2] = -w * w * sin(w * s); break;
    default: b[0] = b[1] = b[2] = NAN; break;
    }
}

/* per-particle mapping table: [12][n] alpha, alpha_x, alpha_y, alpha_xx,
 * alpha_xy, alpha_yy, beta, beta_x, beta_y, beta_xx, beta_xy, beta_yy of
 * every point, for maps of kind ORC_MAP_PER_PARTICLE (set before the calls) */
static const double* g_orc_pp = NULL;
static int64_t g_orc_pp_n = 0;

void orc_set_per_particle(const double* pp, int64_t n)
{
    g_orc_pp = pp;
    g_orc_pp_n = pp ? n : 0;
}

/* real instantiation of the mapping coefficients */
#define ORC_T double
#define ORC_SQRT sqrt
#define ORC_FN(x) orc_r_##x
#include "orc_map_impl.h"
#undef ORC_T
#undef ORC_SQRT
#undef ORC_FN

/* complex instantiation (complex-step derivative with respect to a coefficient) */
#define ORC_T double complex
#define ORC_SQRT csqrt
#define ORC_FN(x) orc_c_##x
#include "orc_map_impl.h"
#undef ORC_T
#undef ORC_SQRT
#undef ORC_FN

/* ------------------------------------------------------------- kernels */

/* Kernel value w(r) and derivative dw/dr.
 *  Wendland C2 with support R:  w = C (1-q)^4 (1+4q), q = r/R,
 *    C = 7/(pi R^2) in 2-D, 21/(2 pi R^3) in 3-D (unit integral).
 *  Cubic spline (paper Sec. 3.1) with smoothing length l = R/2 (r_e = 2 l):
 *    w = a_d [1 - 3/2 s^2 + 3/4 s^3]  (0 <= s <= 1)
 *        a_d [1/4 (2 - s)^3]          (1 <= s <= 2),   s = r/l,
 *    a_d = 10/(7 pi l^2) in 2-D, 1/(pi l^3) in 3-D.                          */
void orc_kernel_eval(int kernel, int dim, double R, double r, double* w, double* dwdr)
{
    if (kernel == ORC_K_WENDLAND) {
        double C = (dim == 2) ? 7.0 / (M_PI * R * R) : 21.0 / (2.0 * M_PI * R * R * R);
        double q = r / R;
        if (q >= 1.0) { *w = 0.0; *dwdr = 0.0; return; }
        double a = 1.0 - q;
        *w = C * a * a * a * a * (1.0 + 4.0 * q);
        *dwdr = C * (-20.0 * q * a * a * a) / R;
    } else {
        double l = 0.5 * R;
        double ad = (dim == 2) ? 10.0 / (7.0 * M_PI * l * l) : 1.0 / (M_PI * l * l * l);
        double s = r / l;
        if (s <= 1.0) {
            *w = ad * (1.0 - 1.5 * s * s + 0.75 * s * s * s);
            *dwdr = ad * (-3.0 * s + 2.25 * s * s) / l;
        } else if (s < 2.0) {
            double t = 2.0 - s;
            *w = ad * 0.25 * t * t * t;
            *dwdr = ad * (-0.75 * t * t) / l;
        } else {
            *w = 0.0; *dwdr = 0.0;
        }
    }
}

/* ------------------------------------------------------------ linear algebra */

/* Solve A X = B by Gaussian elimination with partial pivoting.  A is n x n
 * (row-major, overwritten), B is n x nrhs (row-major, overwritten with X).
 * Returns 1 if a pivot is not larger than tol * max|A| (singular), else 0. */
static int orc_gepp(int n, double* A, int nrhs, double* B, double tol)
{
    double scale = 0.0;
    for (int k = 0; k < n * n; ++k) {
        if (!isfinite(A[k])) return 1;
        if (fabs(A[k]) > scale) scale = fabs(A[k]);
    }
    if (scale == 0.0) return 1;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (!(fabs(A[piv * n + c]) > tol * scale)) return 1;
        if (piv != c) {
            for (int k = 0; k < n; ++k) { double t = A[c * n + k]; A[c * n + k] = A[piv * n + k]; A[piv * n + k] = t; }
            for (int k = 0; k < nrhs; ++k) { double t = B[c * nrhs + k]; B[c * nrhs + k] = B[piv * nrhs + k]; B[piv * nrhs + k] = t; }
        }
        for (int r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            if (f == 0.0) continue;
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            for (int k = 0; k < nrhs; ++k) B[r * nrhs + k] -= f * B[c * nrhs + k];
        }
    }
    for (int c = n - 1; c >= 0; --c) {
        for (int k = 0; k < nrhs; ++k) {
            double s = B[c * nrhs + k];
            for (int j = c + 1; j < n; ++j) s -= A[c * n + j] * B[j * nrhs + k];
            B[c * nrhs + k] = s / A[c * n + c];
        }
    }
    return 0;
}

/* ------------------------------------------------------------ neighbours */

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* The neighbour test of Eq. SPH_neighbor_set, evaluated left to right. */
static int orc_is_neighbor(int dim, int64_t n, const double* pos, int64_t i, int64_t j, double R2)
{
    double dx = pos[j] - pos[i];
    double dy = pos[n + j] - pos[n + i];
    double d2 = dx * dx;
    d2 = d2 + dy * dy;
    if (dim == 3) {
        double dz = pos[2 * n + j] - pos[2 * n + i];
        d2 = d2 + dz * dz;
    }
    return d2 < R2;
}

typedef struct {
    int dim;
    int64_t n;
    double lo[3], c;          /* bucket origin and size (2 R: slack for rounding) */
    int64_t nb[3];
    int64_t* start;           /* bucket -> first index into `idx` */
    int32_t* idx;             /* particle indices grouped by bucket */
} orc_grid;

static int64_t grid_coord(double v, double lo, double c, int64_t nb)
{
    double t = floor((v - lo) / c);
    if (!(t >= 0.0)) return 0;            /* also catches NaN */
    if (t >= (double)(nb - 1)) return nb - 1;
    return (int64_t)t;
}

static int orc_grid_build(orc_grid* g, int dim, int64_t n, const double* pos, double R)
{
    g->dim = dim; g->n = n; g->c = 2.0 * R;
    for (int a = 0; a < 3; ++a) { g->lo[a] = 0.0; g->nb[a] = 1; }
    for (int a = 0; a < dim; ++a) {
        double mn = INFINITY, mx = -INFINITY;
        for (int64_t i = 0; i < n; ++i) {
            double v = pos[a * n + i];
            if (isfinite(v)) { if (v < mn) mn = v; if (v > mx) mx = v; }
        }
        if (!(mn <= mx)) { mn = 0.0; mx = 0.0; }
        g->lo[a] = mn;
        g->nb[a] = (int64_t)floor((mx - mn) / g->c) + 1;
        if (g->nb[a] > 4096) g->nb[a] = 4096;       /* coarser buckets stay correct */
    }
    int64_t nbk = g->nb[0] * g->nb[1] * g->nb[2];
    g->start = (int64_t*)calloc((size_t)nbk + 1, sizeof(int64_t));
    g->idx = (int32_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t* key = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!g->start || !g->idx || !key) { free(key); return 1; }
    for (int64_t i = 0; i < n; ++i) {
        int64_t k[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) k[a] = grid_coord(pos[a * n + i], g->lo[a], g->c, g->nb[a]);
        key[i] = (k[0] * g->nb[1] + k[1]) * g->nb[2] + k[2];
        g->start[key[i] + 1]++;
    }
    for (int64_t b = 0; b < nbk; ++b) g->start[b + 1] += g->start[b];
    int64_t* fill = (int64_t*)malloc((size_t)(nbk > 0 ? nbk : 1) * sizeof(int64_t));
    if (!fill) { free(key); return 1; }
    for (int64_t b = 0; b < nbk; ++b) fill[b] = g->start[b];
    for (int64_t i = 0; i < n; ++i) g->idx[fill[key[i]]++] = (int32_t)i;
    free(fill);
    free(key);
    return 0;
}

static void orc_grid_free(orc_grid* g) { free(g->start); free(g->idx); }

/* Neighbour indices of particle i (ascending), written to out; returns count.
 * out may be NULL (count only).  brute != 0 scans every particle. */
static int64_t orc_row(const orc_grid* g, const double* pos, int64_t i, double R2, int brute,
                       int32_t* out, int32_t* tmp, int64_t tmpcap)
{
    int dim = g->dim;
    int64_t n = g->n;
    int64_t cnt = 0;
    if (brute) {
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            if (orc_is_neighbor(dim, n, pos, i, j, R2)) { if (out) out[cnt] = (int32_t)j; cnt++; }
        }
        return cnt;
    }
    int64_t k[3] = {0, 0, 0};
    for (int a = 0; a < dim; ++a) k[a] = grid_coord(pos[a * n + i], g->lo[a], g->c, g->nb[a]);
    int64_t ncand = 0;
    for (int64_t b0 = k[0] - 1; b0 <= k[0] + 1; ++b0) {
        if (b0 < 0 || b0 >= g->nb[0]) continue;
        for (int64_t b1 = k[1] - 1; b1 <= k[1] + 1; ++b1) {
            if (b1 < 0 || b1 >= g->nb[1]) continue;
            for (int64_t b2 = k[2] - 1; b2 <= k[2] + 1; ++b2) {
                if (b2 < 0 || b2 >= g->nb[2]) continue;
                int64_t bk = (b0 * g->nb[1] + b1) * g->nb[2] + b2;
                for (int64_t p = g->start[bk]; p < g->start[bk + 1]; ++p) {
                    int64_t j = g->idx[p];
                    if (j == i) continue;
                    if (orc_is_neighbor(dim, n, pos, i, j, R2)) {
                        if (ncand < tmpcap) tmp[ncand] = (int32_t)j;
                        ncand++;
                    }
                }
            }
        }
    }
    if (ncand > tmpcap) return -ncand;     /* caller retries with more room */
    qsort(tmp, (size_t)ncand, sizeof(int32_t), cmp_i32);
    if (out) memcpy(out, tmp, (size_t)ncand * sizeof(int32_t));
    return ncand;
}

int64_t orc_neighbors(int dim, int64_t n, const double* pos, double R, int64_t nrows,
                      const int64_t* rows, int brute, int64_t* row_ptr, int32_t* col, int64_t cap)
{
    if ((dim != 2 && dim != 3) || n < 0 || !(R > 0)) return -1;
    const double R2 = R * R;
    orc_grid g;
    memset(&g, 0, sizeof g);
    if (orc_grid_build(&g, dim, n, pos, R)) { orc_grid_free(&g); return -2; }
    int64_t nr = rows ? nrows : n;
    int64_t bad = 0;
    /* pass 1: counts */
    #pragma omp parallel reduction(+:bad)
    {
        int64_t tcap = 4096;
        int32_t* tmp = (int32_t*)malloc((size_t)tcap * sizeof(int32_t));
        #pragma omp for schedule(dynamic, 256)
        for (int64_t r = 0; r < nr; ++r) {
            int64_t i = rows ? rows[r] : r;
            int64_t c = orc_row(&g, pos, i, R2, brute, NULL, tmp, tcap);
            while (c < 0) {
                tcap = -c * 2;
                tmp = (int32_t*)realloc(tmp, (size_t)tcap * sizeof(int32_t));
                c = orc_row(&g, pos, i, R2, brute, NULL, tmp, tcap);
            }
            row_ptr[r + 1] = c;
        }
        free(tmp);
    }
    (void)bad;
    row_ptr[0] = 0;
    for (int64_t r = 0; r < nr; ++r) row_ptr[r + 1] += row_ptr[r];
    int64_t nnz = row_ptr[nr];
    if (col && cap >= nnz) {
        #pragma omp parallel
        {
            int64_t tcap = 4096;
            int32_t* tmp = (int32_t*)malloc((size_t)tcap * sizeof(int32_t));
            #pragma omp for schedule(dynamic, 256)
            for (int64_t r = 0; r < nr; ++r) {
                int64_t i = rows ? rows[r] : r;
                int64_t need = row_ptr[r + 1] - row_ptr[r];
                if (need > tcap) { tcap = need; tmp = (int32_t*)realloc(tmp, (size_t)tcap * sizeof(int32_t)); }
                orc_row(&g, pos, i, R2, brute, col + row_ptr[r], tmp, tcap);
            }
            free(tmp);
        }
    }
    orc_grid_free(&g);
    return nnz;
}

/* ------------------------------------------------------ per-particle SPH(2) */

typedef struct {
    int dim, m;
    int64_t n;
    const double* pos;
    const double* vol;
    int kernel;
    double R;
    orc_map map;
    int grad_order;
} orc_ctx;

/* per-thread scratch, sized for the largest neighbour count */
typedef struct {
    int64_t cap;
    double *r, *gw, *gt, *q, *p, *F, *phiij;
} orc_scratch;

static int scratch_reserve(orc_scratch* s, int64_t deg)
{
    if (deg <= s->cap) return 0;
    int64_t c = deg + 64;
    free(s->r); free(s->gw); free(s->gt); free(s->q); free(s->p); free(s->F); free(s->phiij);
    s->r = malloc((size_t)c * 3 * sizeof(double));
    s->gw = malloc((size_t)c * 3 * sizeof(double));
    s->gt = malloc((size_t)c * 3 * sizeof(double));
    s->q = malloc((size_t)c * 6 * sizeof(double));
    s->p = malloc((size_t)c * 6 * sizeof(double));
    s->F = malloc((size_t)c * sizeof(double));
    s->phiij = malloc((size_t)c * sizeof(double));
    s->cap = c;
    return !(s->r && s->gw && s->gt && s->q && s->p && s->F && s->phiij);
}

static void scratch_free(orc_scratch* s)
{
    free(s->r); free(s->gw); free(s->gt); free(s->q); free(s->p); free(s->F); free(s->phiij);
    memset(s, 0, sizeof *s);
}

/* Monomials q of a difference vector: 2-D (x, z): [x^2, z^2, xz];
 * 3-D: [x^2, y^2, z^2, xy, xz, yz]. */
static void orc_q(int dim, const double* r, double* q)
{
    if (dim == 2) {
        q[0] = r[0] * r[0]; q[1] = r[1] * r[1]; q[2] = r[0] * r[1];
    } else {
        q[0] = r[0] * r[0]; q[1] = r[1] * r[1]; q[2] = r[2] * r[2];
        q[3] = r[0] * r[1]; q[4] = r[0] * r[2]; q[5] = r[1] * r[2];
    }
}

/* Geometry-only part for particle i: neighbours' difference vectors, kernel
 * gradients, L_i, corrected gradients, Q_i, p_ij, F_ij, and M_i.
 * Returns the flag bits (0 when usable). */
typedef struct {
    double L[9];       /* L_i (d x d, row-major) */
    double Q[18];      /* Q_i (m x d, row-major) */
    double M[36];      /* M_i (m x m, row-major) */
} orc_geom;

static int orc_particle_geometry(const orc_ctx* c, int64_t i, const int32_t* nb, int64_t deg,
                                 orc_scratch* s, orc_geom* G)
{
    const int d = c->dim, m = c->m;
    const int64_t n = c->n;
    int flags = 0;
    for (int a = 0; a < d; ++a) if (!isfinite(c->pos[a * n + i])) flags |= ORC_F_NONFINITE;
    if (!isfinite(c->vol[i])) flags |= ORC_F_NONFINITE;
    if (deg < d + m) flags |= ORC_F_FEW;
    if (flags) return flags;
    /* difference vectors and kernel gradients grad w_ij = -(dw/dr) r_ij / |r_ij| */
    for (int64_t k = 0; k < deg; ++k) {
        int64_t j = nb[k];
        double d2 = 0.0;
        for (int a = 0; a < d; ++a) {
            s->r[3 * k + a] = c->pos[a * n + j] - c->pos[a * n + i];
            d2 += s->r[3 * k + a] * s->r[3 * k + a];
        }
        if (!isfinite(c->vol[j]) || !isfinite(d2)) flags |= ORC_F_NONFINITE;
        if (d2 == 0.0) { flags |= ORC_F_DUPLICATE; continue; }
        double rr = sqrt(d2), w, dw;
        orc_kernel_eval(c->kernel, d, c->R, rr, &w, &dw);
        for (int a = 0; a < d; ++a) s->gw[3 * k + a] = -dw * s->r[3 * k + a] / rr;
        s->F[k] = d2;     /* keep |r|^2 for the F_ij denominator */
        orc_q(d, s->r + 3 * k, s->q + 6 * k);
    }
    if (flags) return flags;
    /* A_i = sum_j V_j grad w_ij (x) r_ij, L_i = A_i^-1 */
    double A[9] = {0}, Linv[9] = {0};
    for (int64_t k = 0; k < deg; ++k) {
        double V = c->vol[nb[k]];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) A[a * d + b] += V * s->gw[3 * k + a] * s->r[3 * k + b];
    }
    for (int a = 0; a < d; ++a) Linv[a * d + a] = 1.0;
    if (orc_gepp(d, A, d, Linv, ORC_PIVOT_TOL)) return ORC_F_SINGULAR_A;
    memcpy(G->L, Linv, sizeof(double) * d * d);
    /* corrected kernel gradients */
    for (int64_t k = 0; k < deg; ++k)
        for (int a = 0; a < d; ++a) {
            double t = 0.0;
            for (int b = 0; b < d; ++b) t += G->L[a * d + b] * s->gw[3 * k + b];
            s->gt[3 * k + a] = t;
        }
    /* Q_i = sum_k V_k q_ik (L_i grad w_ik)^T */
    memset(G->Q, 0, sizeof G->Q);
    for (int64_t k = 0; k < deg; ++k) {
        double V = c->vol[nb[k]];
        for (int mm = 0; mm < m; ++mm)
            for (int a = 0; a < d; ++a) G->Q[mm * d + a] += V * s->q[6 * k + mm] * s->gt[3 * k + a];
    }
    /* p_ij = q_ij - Q_i r_ij;  F_ij = r_ij . (L_i grad w_ij) / |r_ij|^4 */
    for (int64_t k = 0; k < deg; ++k) {
        double d2 = s->F[k];
        double rg = 0.0;
        for (int a = 0; a < d; ++a) rg += s->r[3 * k + a] * s->gt[3 * k + a];
        s->F[k] = rg / (d2 * d2);
        for (int mm = 0; mm < m; ++mm) {
            double t = 0.0;
            for (int a = 0; a < d; ++a) t += G->Q[mm * d + a] * s->r[3 * k + a];
            s->p[6 * k + mm] = s->q[6 * k + mm] - t;
        }
    }
    /* M_i = sum_j V_j F_ij q_ij p_ij^T */
    memset(G->M, 0, sizeof G->M);
    for (int64_t k = 0; k < deg; ++k) {
        double VF = c->vol[nb[k]] * s->F[k];
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) G->M[a * m + b] += VF * s->q[6 * k + a] * s->p[6 * k + b];
    }
    return 0;
}

/* Field part for particle i given the phi_ij values in s->phiij; writes one
 * ORC_REC record.  Returns flag bits. */
/* Physical derivatives at particle i from projected ones (Sec. 2.1): the
 * gradient J grad^ (Eq. grad_VCT), the Laplacian c_trans . D^ (Eq. lap_VCT)
 * and the Hessian J H^ J^T + (d phi/d z^) (d2 z^) (the chain rule, of which
 * Eq. lap_VCT is the trace).  gh and Hh in the 3-D component order (x, y, z^);
 * fills rec[0:13], rec[25:32]; returns ORC_F_MAP where alpha is not positive. */
static int orc_physical_record(const orc_ctx* c, int64_t i, const double gh[3], double Hh[3][3], double* rec)
{
    const int d = c->dim;
    const int64_t n = c->n;
    double x = c->pos[i], y = (d == 3) ? c->pos[n + i] : 0.0, zh = c->pos[(d - 1) * n + i];
    double Jm[3][3], ct[6], hz[3][3];
    orc_r_map_coeffs(&c->map, d, x, y, zh, i, -1, 0.0, Jm, ct, hz);
    /* the transformation needs alpha > 0 (Sec. 2.1); Jm[2][2] is alpha */
    if (!(Jm[2][2] > 0.0) || !isfinite(Jm[2][2] + Jm[0][2] + Jm[1][2] + ct[0] + hz[0][1])) return ORC_F_MAP;
    double Dhat[6] = {gh[2], Hh[0][0], Hh[1][1], Hh[2][2], Hh[0][2], Hh[1][2]};
    double lap = 0.0;
    for (int k = 0; k < 6; ++k) lap += ct[k] * Dhat[k];
    double gp[3];
    for (int I = 0; I < 3; ++I) {
        double t = 0.0;
        for (int K = 0; K < 3; ++K) t += Jm[I][K] * gh[K];
        gp[I] = t;
    }
    double Hp[3][3];
    for (int I = 0; I < 3; ++I)
        for (int L = 0; L < 3; ++L) {
            double t = 0.0;
            for (int K = 0; K < 3; ++K)
                for (int Mx = 0; Mx < 3; ++Mx) t += Jm[I][K] * Hh[K][Mx] * Jm[L][Mx];
            Hp[I][L] = t + gh[2] * hz[I][L];
        }
    if (d == 2) {
        /* the 2-D plane has no y: drop the y row and column */
        Hp[1][1] = 0.0; Hp[0][1] = Hp[1][0] = Hp[1][2] = Hp[2][1] = 0.0; gp[1] = 0.0;
    }
    rec[0] = gp[0]; rec[1] = gp[1]; rec[2] = gp[2];
    rec[3] = lap;
    rec[4] = Hp[0][1]; rec[5] = Hp[0][2]; rec[6] = Hp[1][2];
    rec[7] = Hp[0][0]; rec[8] = Hp[1][1]; rec[9] = Hp[2][2];
    rec[10] = Hp[0][1]; rec[11] = Hp[0][2]; rec[12] = Hp[1][2];
    for (int k = 0; k < 6; ++k) rec[25 + k] = Dhat[k];
    rec[31] = Hp[0][0] + Hp[1][1] + Hp[2][2];
    return 0;
}

static int orc_particle_field(const orc_ctx* c, int64_t i, const int32_t* nb, int64_t deg,
                              const orc_scratch* s, const orc_geom* G, double* rec)
{
    const int d = c->dim, m = c->m;
    for (int k = 0; k < ORC_REC; ++k) rec[k] = 0.0;
    /* g1_i = sum_j V_j phi_ij L_i grad w_ij */
    double g1[3] = {0, 0, 0};
    for (int64_t k = 0; k < deg; ++k) {
        double V = c->vol[nb[k]];
        for (int a = 0; a < d; ++a) g1[a] += V * s->phiij[k] * s->gt[3 * k + a];
    }
    /* right-hand side sum_j V_j F_ij q_ij (phi_ij - r_ij . g1_i) */
    double b[6] = {0, 0, 0, 0, 0, 0};
    for (int64_t k = 0; k < deg; ++k) {
        double rg = 0.0;
        for (int a = 0; a < d; ++a) rg += s->r[3 * k + a] * g1[a];
        double t = c->vol[nb[k]] * s->F[k] * (s->phiij[k] - rg);
        for (int mm = 0; mm < m; ++mm) b[mm] += t * s->q[6 * k + mm];
    }
    double M[36];
    memcpy(M, G->M, sizeof(double) * m * m);
    if (orc_gepp(m, M, 1, b, ORC_PIVOT_TOL)) return ORC_F_SINGULAR_M;
    double D[6];
    for (int mm = 0; mm < m; ++mm) D[mm] = 2.0 * b[mm];
    /* second-order gradient g1 - 1/2 Q^T D */
    double g2[3];
    for (int a = 0; a < d; ++a) {
        double t = 0.0;
        for (int mm = 0; mm < m; ++mm) t += G->Q[mm * d + a] * D[mm];
        g2[a] = g1[a] - 0.5 * t;
    }
    const double* gsel = (c->grad_order == 1) ? g1 : g2;
    /* embed into 3-D component order (x, y, z^) */
    double gh[3] = {0, 0, 0}, Hh[3][3] = {{0}}, g1e[3] = {0, 0, 0}, g2e[3] = {0, 0, 0}, De[6] = {0};
    if (d == 2) {
        gh[0] = gsel[0]; gh[2] = gsel[1];
        g1e[0] = g1[0]; g1e[2] = g1[1]; g2e[0] = g2[0]; g2e[2] = g2[1];
        Hh[0][0] = D[0]; Hh[2][2] = D[1]; Hh[0][2] = Hh[2][0] = 0.5 * D[2];
        De[0] = D[0]; De[2] = D[1]; De[4] = D[2];
    } else {
        for (int a = 0; a < 3; ++a) { gh[a] = gsel[a]; g1e[a] = g1[a]; g2e[a] = g2[a]; }
        Hh[0][0] = D[0]; Hh[1][1] = D[1]; Hh[2][2] = D[2];
        Hh[0][1] = Hh[1][0] = 0.5 * D[3];
        Hh[0][2] = Hh[2][0] = 0.5 * D[4];
        Hh[1][2] = Hh[2][1] = 0.5 * D[5];
        for (int k = 0; k < 6; ++k) De[k] = D[k];
    }
    for (int a = 0; a < 3; ++a) { rec[13 + a] = g1e[a]; rec[16 + a] = g2e[a]; }
    for (int k = 0; k < 6; ++k) rec[19 + k] = De[k];
    return orc_physical_record(c, i, gh, Hh, rec);
}

static void nan_record(double* rec) { for (int k = 0; k < ORC_REC; ++k) rec[k] = NAN; }

static void ctx_init(orc_ctx* c, int dim, int64_t n, const double* pos, const double* vol,
                     int kernel, double R, int map_kind, double Hhat, double H, double dmin,
                     double eps, int nterms, const double* terms, int grad_order)
{
    c->dim = dim; c->m = (dim == 2) ? 3 : 6; c->n = n; c->pos = pos; c->vol = vol;
    c->kernel = kernel; c->R = R; c->grad_order = grad_order;
    c->map.kind = map_kind; c->map.Hhat = Hhat; c->map.H = H; c->map.dmin = dmin;
    c->map.eps = eps; c->map.nterms = nterms; c->map.terms = terms;
}

int orc_sph2(int dim, int64_t n, const double* pos, const double* vol, int nf, const double* phi,
             int kernel, double R, int map_kind, double Hhat, double H, double dmin, double eps,
             int nterms, const double* terms, int grad_order,
             int64_t nrows, const int64_t* rows, const int64_t* row_ptr, const int32_t* col,
             double* out, uint8_t* flags)
{
    if ((dim != 2 && dim != 3) || n < 0 || nf < 0 || !(R > 0)) return -1;
    orc_ctx c;
    ctx_init(&c, dim, n, pos, vol, kernel, R, map_kind, Hhat, H, dmin, eps, nterms, terms, grad_order);
    #pragma omp parallel
    {
        orc_scratch s;
        memset(&s, 0, sizeof s);
        #pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t i = rows ? rows[r] : r;
            const int32_t* nb = col + row_ptr[r];
            int64_t deg = row_ptr[r + 1] - row_ptr[r];
            double* o = out + (size_t)r * nf * ORC_REC;
            int fl = scratch_reserve(&s, deg) ? ORC_F_NONFINITE : 0;
            orc_geom G;
            if (!fl) fl = orc_particle_geometry(&c, i, nb, deg, &s, &G);
            for (int f = 0; f < nf; ++f) {
                double* rec = o + (size_t)f * ORC_REC;
                int ff = fl;
                if (!ff) {
                    const double* ph = phi + (size_t)f * n;
                    for (int64_t k = 0; k < deg; ++k) s.phiij[k] = ph[nb[k]] - ph[i];
                    ff = orc_particle_field(&c, i, nb, deg, &s, &G, rec);
                }
                if (ff) nan_record(rec);
                fl |= ff;
            }
            if (flags) flags[r] = (uint8_t)fl;
        }
        scratch_free(&s);
    }
    return 0;
}

/* Adjoint of the physical Laplacian with respect to the field, at sampled
 * particles k:  dphi_k = sum_i u_i d(lap_i)/d(phi_k), i over S_k and k itself.
 * d(lap_i)/d(phi_k) is the Laplacian at i of the unit field e_k (the operator
 * is linear in phi), evaluated with the full per-particle computation.
 * row_ptr/col is the CSR of *all* particles. */
int orc_adjoint_dphi(int dim, int64_t n, const double* pos, const double* vol, int kernel, double R,
                     int map_kind, double Hhat, double H, double dmin, double eps, int nterms,
                     const double* terms, int grad_order, const int64_t* row_ptr, const int32_t* col,
                     const double* u, int64_t nk, const int64_t* ks, double* dphi)
{
    if ((dim != 2 && dim != 3) || n < 0 || !(R > 0)) return -1;
    orc_ctx c;
    ctx_init(&c, dim, n, pos, vol, kernel, R, map_kind, Hhat, H, dmin, eps, nterms, terms, grad_order);
    int status = 0;
    #pragma omp parallel
    {
        orc_scratch s;
        memset(&s, 0, sizeof s);
        double rec[ORC_REC];
        #pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nk; ++t) {
            int64_t k = ks ? ks[t] : t;
            double acc = 0.0;
            int64_t nkdeg = row_ptr[k + 1] - row_ptr[k];
            for (int64_t e = -1; e < nkdeg; ++e) {
                int64_t i = (e < 0) ? k : col[row_ptr[k] + e];
                const int32_t* nb = col + row_ptr[i];
                int64_t deg = row_ptr[i + 1] - row_ptr[i];
                if (scratch_reserve(&s, deg)) { acc = NAN; break; }
                orc_geom G;
                int fl = orc_particle_geometry(&c, i, nb, deg, &s, &G);
                if (fl) { acc = NAN; continue; }
                for (int64_t q = 0; q < deg; ++q)
                    s.phiij[q] = (nb[q] == k ? 1.0 : 0.0) - (i == k ? 1.0 : 0.0);
                fl = orc_particle_field(&c, i, nb, deg, &s, &G, rec);
                if (fl) { acc = NAN; continue; }
                acc += u[i] * rec[3];
            }
            dphi[t] = acc;
        }
        scratch_free(&s);
    }
    return status;
}

/* Sensitivity of the physical Laplacian to bathymetry coefficient t at fixed
 * projected positions, by the complex-step derivative of c_trans:
 *   dtheta_t = sum_i u_i (d c_trans_i / d coef_t) . Dhat_i
 * Dhat (n x 6) holds the projected derivative vectors [dz^, xx, yy, zz, xz, yz].
 * The sum runs over particles in index order with Kahan compensation.       */
int orc_dtheta(int dim, int64_t n, const double* pos, int map_kind, double Hhat, double H,
               double dmin, double eps, int nterms, const double* terms, const double* u,
               const double* Dhat, int nt, const int32_t* tlist, double* dtheta)
{
    orc_map mp;
    mp.kind = map_kind; mp.Hhat = Hhat; mp.H = H; mp.dmin = dmin; mp.eps = eps;
    mp.nterms = nterms; mp.terms = terms;
    const double hstep = 1e-30;
    #pragma omp parallel for schedule(static, 1)
    for (int tt = 0; tt < nt; ++tt) {
        int t = tlist[tt];
        double sum = 0.0, comp = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double x = pos[i], y = (dim == 3) ? pos[n + i] : 0.0, zh = pos[(dim - 1) * n + i];
            double complex Jm[3][3], ct[6], hz[3][3];
            orc_c_map_coeffs(&mp, dim, x, y, zh, i, t, hstep * _Complex_I, Jm, ct, hz);
            double v = 0.0;
            for (int k = 0; k < 6; ++k) v += cimag(ct[k]) / hstep * Dhat[6 * i + k];
            double yv = u[i] * v - comp;
            double tv = sum + yv;
            comp = (tv - sum) - yv;
            sum = tv;
        }
        dtheta[tt] = sum;
    }
    return 0;
}

/* Mapping coefficients at given points (for tests): out per point =
 * [J (9, row-major), c_trans (6), d2z^ (9)] and, with t >= 0, the complex-step
 * derivative of the same 24 numbers with respect to coefficient t.          */
int orc_map_eval(int dim, int64_t np, const double* x, const double* y, const double* zh,
                 int map_kind, double Hhat, double H, double dmin, double eps, int nterms,
                 const double* terms, int t, double* out)
{
    orc_map mp;
    mp.kind = map_kind; mp.Hhat = Hhat; mp.H = H; mp.dmin = dmin; mp.eps = eps;
    mp.nterms = nterms; mp.terms = terms;
    for (int64_t p = 0; p < np; ++p) {
        double* o = out + 24 * p;
        if (t < 0) {
            double Jm[3][3], ct[6], hz[3][3];
            orc_r_map_coeffs(&mp, dim, x[p], y ? y[p] : 0.0, zh[p], p, -1, 0.0, Jm, ct, hz);
            for (int a = 0; a < 9; ++a) o[a] = Jm[a / 3][a % 3];
            for (int a = 0; a < 6; ++a) o[9 + a] = ct[a];
            for (int a = 0; a < 9; ++a) o[15 + a] = hz[a / 3][a % 3];
        } else {
            const double hstep = 1e-30;
            double complex Jm[3][3], ct[6], hz[3][3];
            orc_c_map_coeffs(&mp, dim, x[p], y ? y[p] : 0.0, zh[p], p, t, hstep * _Complex_I, Jm, ct, hz);
            for (int a = 0; a < 9; ++a) o[a] = cimag(Jm[a / 3][a % 3]) / hstep;
            for (int a = 0; a < 6; ++a) o[9 + a] = cimag(ct[a]) / hstep;
            for (int a = 0; a < 9; ++a) o[15 + a] = cimag(hz[a / 3][a % 3]) / hstep;
        }
    }
    return 0;
}

/* alpha, beta and derivatives at given points (for tests), 12 per point. */
int orc_alpha_beta(int dim, int64_t np, const double* x, const double* y, int map_kind, double Hhat,
                   double H, double dmin, double eps, int nterms, const double* terms, double* out)
{
    orc_map mp;
    mp.kind = map_kind; mp.Hhat = Hhat; mp.H = H; mp.dmin = dmin; mp.eps = eps;
    mp.nterms = nterms; mp.terms = terms;
    for (int64_t p = 0; p < np; ++p)
        orc_r_alpha_beta(&mp, dim, x[p], y ? y[p] : 0.0, p, -1, 0.0, out + 12 * p);
    return 0;
}

int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Thread count of the following parallel regions (timing only; n <= 0 keeps it). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ================================================= ISPH pressure step (Sec. 3.3) */

/* Weights of the physical Laplacian (Eq. lap_VCT with the SPH(2) second
 * derivatives of Eq. sec_SPH2): lap_i(phi) = sum_j W_ij (phi_j - phi_i).  The
 * operator is linear in the differences phi_ij, so W_ij is the operator applied
 * to the field whose differences are phi_ik = delta_kj.  The steps are those of
 * orc_particle_field, taken for every such unit field of the row at once:
 *   g1(e_j)  = V_j L_i grad w_ij                                   (Eq. gra_1st)
 *   b(e_j)   = V_j F_ij q_ij - (sum_k V_k F_ik q_ik r_ik^T) g1(e_j)
 *   D(e_j)   = 2 M_i^-1 b(e_j)                                     (Eq. sec_SPH2)
 *   g2(e_j)  = g1(e_j) - 1/2 Q_i^T D(e_j)
 *   W_ij     = c_trans . D^(e_j)                                   (Eq. lap_VCT)
 * W has the layout of col (row r of the CSR holds the weights of rows[r]).
 * Flagged particles get NaN weights. */
int orc_lap_weights(int dim, int64_t n, const double* pos, const double* vol, int kernel, double R,
                    int map_kind, double Hhat, double H, double dmin, double eps, int nterms,
                    const double* terms, int grad_order, int64_t nrows, const int64_t* rows,
                    const int64_t* row_ptr, const int32_t* col, double* W, uint8_t* flags)
{
    if ((dim != 2 && dim != 3) || n < 0 || !(R > 0)) return -1;
    orc_ctx c;
    ctx_init(&c, dim, n, pos, vol, kernel, R, map_kind, Hhat, H, dmin, eps, nterms, terms, grad_order);
    const int d = dim, m = c.m;
    #pragma omp parallel
    {
        orc_scratch s;
        memset(&s, 0, sizeof s);
        int64_t bcap = 0;
        double* B = NULL;
        #pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t i = rows ? rows[r] : r;
            const int32_t* nb = col + row_ptr[r];
            int64_t deg = row_ptr[r + 1] - row_ptr[r];
            double* w = W + row_ptr[r];
            int fl = scratch_reserve(&s, deg) ? ORC_F_NONFINITE : 0;
            if (deg > bcap) { bcap = deg + 64; free(B); B = (double*)malloc((size_t)bcap * 6 * sizeof(double)); }
            orc_geom G;
            if (!fl) fl = orc_particle_geometry(&c, i, nb, deg, &s, &G);
            /* C_i = sum_k V_k F_ik q_ik r_ik^T (m x d) */
            double Cm[18] = {0};
            if (!fl) {
                for (int64_t k = 0; k < deg; ++k) {
                    double VF = c.vol[nb[k]] * s.F[k];
                    for (int a = 0; a < m; ++a)
                        for (int b = 0; b < d; ++b) Cm[a * d + b] += VF * s.q[6 * k + a] * s.r[3 * k + b];
                }
                /* right-hand sides b(e_j), one column per neighbour (row-major m x deg) */
                for (int64_t j = 0; j < deg; ++j) {
                    double Vj = c.vol[nb[j]];
                    for (int a = 0; a < m; ++a) {
                        double t = 0.0;
                        for (int b = 0; b < d; ++b) t += Cm[a * d + b] * Vj * s.gt[3 * j + b];
                        B[a * deg + j] = Vj * s.F[j] * s.q[6 * j + a] - t;
                    }
                }
                double M[36];
                memcpy(M, G.M, sizeof(double) * m * m);
                if (orc_gepp(m, M, (int)deg, B, ORC_PIVOT_TOL)) fl |= ORC_F_SINGULAR_M;
            }
            double Jm[3][3], ct[6], hz[3][3];
            if (!fl) {
                double x = c.pos[i], y = (d == 3) ? c.pos[n + i] : 0.0, zh = c.pos[(d - 1) * n + i];
                orc_r_map_coeffs(&c.map, d, x, y, zh, i, -1, 0.0, Jm, ct, hz);
                if (!(Jm[2][2] > 0.0) || !isfinite(Jm[2][2] + Jm[0][2] + Jm[1][2] + ct[0] + hz[0][1])) fl |= ORC_F_MAP;
            }
            for (int64_t j = 0; j < deg; ++j) {
                if (fl) { w[j] = NAN; continue; }
                double Vj = c.vol[nb[j]];
                double D[6], g1[3], g2[3];
                for (int a = 0; a < m; ++a) D[a] = 2.0 * B[a * deg + j];
                for (int a = 0; a < d; ++a) {
                    g1[a] = Vj * s.gt[3 * j + a];
                    double t = 0.0;
                    for (int p = 0; p < m; ++p) t += G.Q[p * d + a] * D[p];
                    g2[a] = g1[a] - 0.5 * t;
                }
                const double* gs = (grad_order == 1) ? g1 : g2;
                double Dhat[6];
                if (d == 2) {   /* (x, z): D = [xx, zz, 2xz] */
                    Dhat[0] = gs[1]; Dhat[1] = D[0]; Dhat[2] = 0.0; Dhat[3] = D[1]; Dhat[4] = 0.5 * D[2]; Dhat[5] = 0.0;
                } else {        /* D = [xx, yy, zz, 2xy, 2xz, 2yz] */
                    Dhat[0] = gs[2]; Dhat[1] = D[0]; Dhat[2] = D[1]; Dhat[3] = D[2]; Dhat[4] = 0.5 * D[4]; Dhat[5] = 0.5 * D[5];
                }
                double t = 0.0;
                for (int k = 0; k < 6; ++k) t += ct[k] * Dhat[k];
                w[j] = t;
            }
            if (flags) flags[r] = (uint8_t)fl;
        }
        free(B);
        scratch_free(&s);
    }
    return 0;
}

/* First-order projected gradient <grad^ f>^(1)_i = sum_j V_j f_ij L_i grad w_ij
 * (Eqs. gra_1st, div_1st) of one scalar field at particle i, given its
 * geometry; g[3] in the 3-D component order (2-D: x^, 0, z^). */
static void orc_grad1(const orc_ctx* c, int64_t i, const int32_t* nb, int64_t deg, const orc_scratch* s,
                      const double* f, double g[3])
{
    double t[3] = {0.0, 0.0, 0.0};
    for (int64_t k = 0; k < deg; ++k) {
        double fij = f[nb[k]] - f[i];
        double V = c->vol[nb[k]];
        for (int a = 0; a < c->dim; ++a) t[a] += V * fij * s->gt[3 * k + a];
    }
    g[0] = t[0];
    g[1] = (c->dim == 3) ? t[1] : 0.0;
    g[2] = t[c->dim - 1];
}

/* geometry of particle i for the first-order operators: flags if the state the
 * library would write is NaN there (any geometry flag, a singular M, alpha) */
static int orc_first_order_geometry(const orc_ctx* c, int64_t i, const int32_t* nb, int64_t deg, orc_scratch* s,
                                    double Jm[3][3])
{
    orc_geom G;
    int fl = orc_particle_geometry(c, i, nb, deg, s, &G);
    if (fl) return fl;
    double M[36], b[6] = {0, 0, 0, 0, 0, 0};
    memcpy(M, G.M, sizeof(double) * c->m * c->m);
    if (orc_gepp(c->m, M, 1, b, ORC_PIVOT_TOL)) return ORC_F_SINGULAR_M;
    double ct[6], hz[3][3];
    double x = c->pos[i], y = (c->dim == 3) ? c->pos[c->n + i] : 0.0, zh = c->pos[(c->dim - 1) * c->n + i];
    orc_r_map_coeffs(&c->map, c->dim, x, y, zh, i, -1, 0.0, Jm, ct, hz);
    if (!(Jm[2][2] > 0.0) || !isfinite(Jm[2][2] + Jm[0][2] + Jm[1][2] + ct[0] + hz[0][1])) return ORC_F_MAP;
    return 0;
}

/* Right-hand side of the pressure Poisson equation (Eqs. VCT_ppe, VCT_ppe_w):
 *   rhs_i = rho / dt * div_i + gamma * (rho * jr_i - dens_i) / dt^2
 *   div_i  = sum_{I,K} J_IK <d v_I / d x^_K>^(1)_i     physical divergence of v
 *            through the projected first-order gradients (Eqs. div_1st, jacobi);
 *            v is (dim x n), components along the physical axes
 *   dens_i = rho * (sum_{j in S_i} V_j w_ij + V_i w(0))  numerical density in the
 *            projected space (kernel summation over S_i and i itself)
 *   jr_i   = Jbar_i / J_i of Eq. VCT_ppe_w (1 when jr is NULL, Eq. VCT_ppe)
 * Dirichlet rows (dirichlet[i] != 0) get rhs_i = pbc_i (0 if pbc is NULL).
 * div and dens are written when not NULL; flagged particles get NaN. */
int orc_ppe_rhs(int dim, int64_t n, const double* pos, const double* vol, int kernel, double R, int map_kind,
                double Hhat, double H, double dmin, double eps, int nterms, const double* terms, const double* v,
                double rho, double dt, double gamma, const double* jr, const uint8_t* dirichlet, const double* pbc,
                const int64_t* row_ptr, const int32_t* col, double* rhs, double* div, double* dens)
{
    if ((dim != 2 && dim != 3) || n < 0 || !(R > 0)) return -1;
    orc_ctx c;
    ctx_init(&c, dim, n, pos, vol, kernel, R, map_kind, Hhat, H, dmin, eps, nterms, terms, 2);
    double w0, dw0;
    orc_kernel_eval(kernel, dim, R, 0.0, &w0, &dw0);
    #pragma omp parallel
    {
        orc_scratch s;
        memset(&s, 0, sizeof s);
        #pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            const int32_t* nb = col + row_ptr[i];
            int64_t deg = row_ptr[i + 1] - row_ptr[i];
            double Jm[3][3];
            int fl = scratch_reserve(&s, deg) ? ORC_F_NONFINITE : 0;
            if (!fl) fl = orc_first_order_geometry(&c, i, nb, deg, &s, Jm);
            double dv = NAN, ds = NAN;
            if (!fl) {
                dv = 0.0;
                for (int I = 0; I < dim; ++I) {
                    double g[3];
                    orc_grad1(&c, i, nb, deg, &s, v + (size_t)I * n, g);
                    int Ip = (dim == 3) ? I : (I == 0 ? 0 : 2);   /* physical axis of component I */
                    for (int K = 0; K < 3; ++K) dv += Jm[Ip][K] * g[K];
                }
                double sw = c.vol[i] * w0;
                for (int64_t k = 0; k < deg; ++k) {
                    int64_t j = nb[k];
                    double d2 = 0.0;
                    for (int a = 0; a < dim; ++a) {
                        double t = c.pos[a * n + j] - c.pos[a * n + i];
                        d2 += t * t;
                    }
                    double wv, dwv;
                    orc_kernel_eval(kernel, dim, R, sqrt(d2), &wv, &dwv);
                    sw += c.vol[j] * wv;
                }
                ds = rho * sw;
            }
            if (div) div[i] = dv;
            if (dens) dens[i] = ds;
            double jri = jr ? jr[i] : 1.0;
            rhs[i] = (dirichlet && dirichlet[i]) ? (pbc ? pbc[i] : 0.0)
                                                 : rho / dt * dv + gamma * (rho * jri - ds) / (dt * dt);
        }
        scratch_free(&s);
    }
    return 0;
}

/* Corrector (Sec. 3.3): v_out = v* - dt / rho * J <grad^ p>^(1) (Eqs. gra_1st,
 * grad_VCT), v and v_out (dim x n) along the physical axes. */
int orc_ppe_correct(int dim, int64_t n, const double* pos, const double* vol, int kernel, double R, int map_kind,
                    double Hhat, double H, double dmin, double eps, int nterms, const double* terms,
                    const double* p, const double* vstar, double rho, double dt, const int64_t* row_ptr,
                    const int32_t* col, double* vout)
{
    if ((dim != 2 && dim != 3) || n < 0 || !(R > 0)) return -1;
    orc_ctx c;
    ctx_init(&c, dim, n, pos, vol, kernel, R, map_kind, Hhat, H, dmin, eps, nterms, terms, 2);
    #pragma omp parallel
    {
        orc_scratch s;
        memset(&s, 0, sizeof s);
        #pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            const int32_t* nb = col + row_ptr[i];
            int64_t deg = row_ptr[i + 1] - row_ptr[i];
            double Jm[3][3];
            int fl = scratch_reserve(&s, deg) ? ORC_F_NONFINITE : 0;
            if (!fl) fl = orc_first_order_geometry(&c, i, nb, deg, &s, Jm);
            double g[3] = {NAN, NAN, NAN}, gp[3] = {NAN, NAN, NAN};
            if (!fl) {
                orc_grad1(&c, i, nb, deg, &s, p, g);
                for (int I = 0; I < 3; ++I) {
                    double t = 0.0;
                    for (int K = 0; K < 3; ++K) t += Jm[I][K] * g[K];
                    gp[I] = t;
                }
            }
            for (int I = 0; I < dim; ++I) {
                int Ip = (dim == 3) ? I : (I == 0 ? 0 : 2);
                vout[(size_t)I * n + i] = vstar[(size_t)I * n + i] - dt / rho * gp[Ip];
            }
        }
        scratch_free(&s);
    }
    return 0;
}

/* A x on the pressure system: sum_j W_ij (x_j - x_i) on ordinary rows, x_i on
 * Dirichlet rows; each row summed in its own order. */
static void orc_ppe_matvec(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* W,
                           const uint8_t* dirichlet, const double* x, double* y)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (dirichlet && dirichlet[i]) { y[i] = x[i]; continue; }
        double t = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) t += W[e] * (x[col[e]] - x[i]);
        y[i] = t;
    }
}

static double orc_dot(int64_t n, const double* a, const double* b)
{
    double t = 0.0;
    for (int64_t i = 0; i < n; ++i) t += a[i] * b[i];
    return t;
}

/* Solve the pressure system A x = b by BiCGSTAB (van der Vorst, 1992) with the
 * Jacobi preconditioner on the right (diag_i = -sum_j W_ij on ordinary rows, 1
 * on Dirichlet rows):
 *   r = b - A x, r^ = r, rho = alpha = omega = 1, v = p = 0
 *   repeat: rho' = (r^, r), beta = (rho'/rho)(alpha/omega),
 *           p = r + beta (p - omega v), p^ = diag^-1 p, v = A p^,
 *           alpha = rho' / (r^, v), s = r - alpha v, s^ = diag^-1 s, t = A s^,
 *           omega = (t, s) / (t, t), x += alpha p^ + omega s^, r = s - omega t
 *   until ||r|| <= tol ||b|| or maxit iterations.
 * x holds the initial guess on entry.  *iters receives the iterations taken and
 * *relres the true relative residual ||b - A x|| / ||b||.  Returns 0, 1 if it
 * stopped without converging, 2 on a breakdown. */
int orc_ppe_bicgstab(int64_t n, const int64_t* row_ptr, const int32_t* col, const double* W,
                     const uint8_t* dirichlet, const double* b, double* x, double tol, int maxit, int* iters,
                     double* relres)
{
    double* buf = (double*)malloc((size_t)(n > 0 ? n : 1) * 9 * sizeof(double));
    if (!buf) return -1;
    double *r = buf, *rh = buf + n, *p = buf + 2 * n, *v = buf + 3 * n, *s = buf + 4 * n, *t = buf + 5 * n;
    double *ph = buf + 6 * n, *sh = buf + 7 * n, *dinv = buf + 8 * n;
    for (int64_t i = 0; i < n; ++i) {
        double dg = 1.0;
        if (!(dirichlet && dirichlet[i])) {
            dg = 0.0;
            for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) dg -= W[e];
        }
        dinv[i] = 1.0 / dg;
    }
    orc_ppe_matvec(n, row_ptr, col, W, dirichlet, x, r);
    for (int64_t i = 0; i < n; ++i) { r[i] = b[i] - r[i]; rh[i] = r[i]; p[i] = 0.0; v[i] = 0.0; }
    double bb = sqrt(orc_dot(n, b, b));
    double rho = 1.0, alpha = 1.0, omega = 1.0;
    int it = 0, status = 1;
    if (sqrt(orc_dot(n, r, r)) <= tol * bb) status = 0;
    while (status == 1 && it < maxit) {
        double rho1 = orc_dot(n, rh, r);
        double beta = (rho1 / rho) * (alpha / omega);
        for (int64_t i = 0; i < n; ++i) { p[i] = r[i] + beta * (p[i] - omega * v[i]); ph[i] = dinv[i] * p[i]; }
        orc_ppe_matvec(n, row_ptr, col, W, dirichlet, ph, v);
        double rv = orc_dot(n, rh, v);
        if (rv == 0.0) { status = 2; break; }
        alpha = rho1 / rv;
        for (int64_t i = 0; i < n; ++i) { s[i] = r[i] - alpha * v[i]; sh[i] = dinv[i] * s[i]; }
        orc_ppe_matvec(n, row_ptr, col, W, dirichlet, sh, t);
        double tt = orc_dot(n, t, t);
        if (tt == 0.0) { status = 2; break; }
        omega = orc_dot(n, t, s) / tt;
        for (int64_t i = 0; i < n; ++i) { x[i] += alpha * ph[i] + omega * sh[i]; r[i] = s[i] - omega * t[i]; }
        rho = rho1;
        ++it;
        if (sqrt(orc_dot(n, r, r)) <= tol * bb) status = 0;
    }
    orc_ppe_matvec(n, row_ptr, col, W, dirichlet, x, t);
    for (int64_t i = 0; i < n; ++i) t[i] = b[i] - t[i];
    *iters = it;
    *relres = bb > 0.0 ? sqrt(orc_dot(n, t, t)) / bb : sqrt(orc_dot(n, t, t));
    free(buf);
    return status;
}

/* ================================================ conventional ISPH operators */

/* The 0th-order models of Sec. 3.1 and the summation pressure gradient of
 * Sec. 3.3, the operators of the ISPH case of Table case_names.  No correction
 * matrix enters.  With r_ij = r_j - r_i and grad w_ij = -w'(r) r_ij / r (the
 * gradient with respect to r_i of w(|r_j - r_i|)), r_ij . grad w_ij / |r_ij|^2
 * is -w'(r) / r, written G below, and grad w_ij = G r_ij. */

/* G = -w'(r)/r of the normalised kernel; NaN at r = 0 */
static double orc_gfac(const orc_ctx* c, double r)
{
    double w, dwdr;
    orc_kernel_eval(c->kernel, c->dim, c->R, r, &w, &dwdr);
    return -dwdr / r;
}

/* projected offset r_ij and its squared length */
static double orc_offset(const orc_ctx* c, int64_t i, int64_t j, double r[3])
{
    double r2 = 0.0;
    for (int a = 0; a < c->dim; ++a) {
        r[a] = c->pos[a * c->n + j] - c->pos[a * c->n + i];
        r2 += r[a] * r[a];
    }
    return r2;
}

/* At particle i, for one field:
 *   <grad^ phi>^(0)_i   = sum_j V_j phi_ij grad w_ij                (Sec. 3.1)
 *   <d2 phi / dx^I dx^J>^(0)_i
 *       = sum_j V_j (c r_ij^I r_ij^J / |r_ij|^2 - delta^IJ)
 *                   (r_ij . grad w_ij / |r_ij|^2) phi_ij,  c = 4 (2-D), 5 (3-D)
 *                                                   (Eq. sec_0th, Espanol & Revenga)
 * then the physical record as for SPH(2).  Record slots 13:19 hold the 0th-order
 * projected gradient (twice) and 19:25 the second derivatives in the SPH(2)
 * vector order with doubled cross terms. */
static int orc_particle_ops0(const orc_ctx* c, int64_t i, const int32_t* nb, int64_t deg, const double* ph,
                             double* rec)
{
    const int d = c->dim;
    const double cc = (d == 2) ? 4.0 : 5.0;
    for (int k = 0; k < ORC_REC; ++k) rec[k] = 0.0;
    double g[3] = {0, 0, 0}, H[3][3] = {{0}};
    for (int64_t k = 0; k < deg; ++k) {
        int64_t j = nb[k];
        double r[3];
        double r2 = orc_offset(c, i, j, r);
        if (!(r2 > 0.0)) return ORC_F_DUPLICATE;
        double G = orc_gfac(c, sqrt(r2));
        double V = c->vol[j], fij = ph[j] - ph[i];
        for (int a = 0; a < d; ++a) g[a] += V * fij * G * r[a];
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b)
                H[a][b] += V * (cc * r[a] * r[b] / r2 - (a == b ? 1.0 : 0.0)) * G * fij;
    }
    /* embed in the 3-D component order (x, y, z^) */
    double gh[3] = {0, 0, 0}, Hh[3][3] = {{0}};
    int ax[3] = {0, 1, 2};
    if (d == 2) { ax[0] = 0; ax[1] = 2; }
    for (int a = 0; a < d; ++a) {
        gh[ax[a]] = g[a];
        for (int b = 0; b < d; ++b) Hh[ax[a]][ax[b]] = H[a][b];
    }
    for (int a = 0; a < 3; ++a) { rec[13 + a] = gh[a]; rec[16 + a] = gh[a]; }
    /* 3-D slot order (xx, yy, zz, 2xy, 2xz, 2yz); 2-D sets leave the y slots zero */
    rec[19] = Hh[0][0]; rec[20] = Hh[1][1]; rec[21] = Hh[2][2];
    rec[22] = 2.0 * Hh[0][1]; rec[23] = 2.0 * Hh[0][2]; rec[24] = 2.0 * Hh[1][2];
    return orc_physical_record(c, i, gh, Hh, rec);
}

/* 0th-order records for nf fields at rows (all particles if rows is NULL),
 * laid out as orc_sph2's; flagged particles get NaN records. */
int orc_ops0(int dim, int64_t n, const double* pos, const double* vol, int nf, const double* phi, int kernel,
             double R, int map_kind, double Hhat, double H, double dmin, double eps, int nterms,
             const double* terms, int64_t nrows, const int64_t* rows, const int64_t* row_ptr, const int32_t* col,
             double* out, uint8_t* flags)
{
    if ((dim != 2 && dim != 3) || n < 0 || nf < 0 || !(R > 0)) return -1;
    orc_ctx c;
    ctx_init(&c, dim, n, pos, vol, kernel, R, map_kind, Hhat, H, dmin, eps, nterms, terms, 2);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows ? rows[r] : r;
        const int32_t* nb = col + row_ptr[r];
        int64_t deg = row_ptr[r + 1] - row_ptr[r];
        int fl = 0;
        for (int f = 0; f < nf; ++f) {
            double* rec = out + ((size_t)r * nf + f) * ORC_REC;
            int ff = orc_particle_ops0(&c, i, nb, deg, phi + (size_t)f * n, rec);
            if (ff) nan_record(rec);
            fl |= ff;
        }
        if (flags) flags[r] = (uint8_t)fl;
    }
    return 0;
}

/* 0th-order Laplacian of Sec. 3.1 (the Brookshaw form), in the projected space:
 *   <lap phi>^(0)_i = 2 sum_j V_j (r_ij . grad w_ij / |r_ij|^2) phi_ij.
 * out [nrows][nf]; NaN where a neighbour sits at zero distance. */
int orc_lap0(int dim, int64_t n, const double* pos, const double* vol, int nf, const double* phi, int kernel,
             double R, int64_t nrows, const int64_t* rows, const int64_t* row_ptr, const int32_t* col, double* out)
{
    if ((dim != 2 && dim != 3) || n < 0 || nf < 0 || !(R > 0)) return -1;
    orc_ctx c;
    ctx_init(&c, dim, n, pos, vol, kernel, R, ORC_MAP_IDENTITY, 1.0, 1.0, 0.0, 0.0, 0, NULL, 2);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows ? rows[r] : r;
        for (int f = 0; f < nf; ++f) {
            const double* ph = phi + (size_t)f * n;
            double t = 0.0;
            for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
                double rv[3];
                double r2 = orc_offset(&c, i, col[k], rv);
                double G = r2 > 0.0 ? orc_gfac(&c, sqrt(r2)) : NAN;
                t += c.vol[col[k]] * G * (ph[col[k]] - ph[i]);
            }
            out[(size_t)r * nf + f] = 2.0 * t;
        }
    }
    return 0;
}

/* Summation pressure gradient (Eq. gra_sum) in the projected space,
 *   <grad^ p>^+_i = rho_i sum_j m_j (p_j / rho_j^2 + p_i / rho_i^2) grad w_ij,
 * with masses m_j = rho_j V_j (rho NULL: rho_j = rho0 for all j), and its
 * physical form J <grad^ p>^+_i (Eq. grad_VCT).  out [nrows][6]: physical
 * (x, y, z) then projected (x^, y^, z^); 2-D sets leave the y slots zero.
 * NaN where alpha is not positive or a neighbour sits at zero distance. */
int orc_grad_sum(int dim, int64_t n, const double* pos, const double* vol, const double* rho, double rho0,
                 const double* p, int kernel, double R, int map_kind, double Hhat, double H, double dmin, double eps,
                 int nterms, const double* terms, int64_t nrows, const int64_t* rows, const int64_t* row_ptr,
                 const int32_t* col, double* out, uint8_t* flags)
{
    if ((dim != 2 && dim != 3) || n < 0 || !(R > 0)) return -1;
    orc_ctx c;
    ctx_init(&c, dim, n, pos, vol, kernel, R, map_kind, Hhat, H, dmin, eps, nterms, terms, 2);
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows ? rows[r] : r;
        double rhoi = rho ? rho[i] : rho0;
        double t[3] = {0, 0, 0};
        int fl = 0;
        for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
            int64_t j = col[k];
            double rv[3];
            double r2 = orc_offset(&c, i, j, rv);
            if (!(r2 > 0.0)) fl |= ORC_F_DUPLICATE;
            double G = orc_gfac(&c, sqrt(r2));
            double rhoj = rho ? rho[j] : rho0;
            double mj = rhoj * c.vol[j];
            double s = mj * (p[j] / (rhoj * rhoj) + p[i] / (rhoi * rhoi));
            for (int a = 0; a < dim; ++a) t[a] += s * G * rv[a];
        }
        double gh[3] = {rhoi * t[0], dim == 3 ? rhoi * t[1] : 0.0, rhoi * t[dim - 1]};
        double x = c.pos[i], y = (dim == 3) ? c.pos[n + i] : 0.0, zh = c.pos[(dim - 1) * n + i];
        double Jm[3][3], ct[6], hz[3][3];
        orc_r_map_coeffs(&c.map, dim, x, y, zh, i, -1, 0.0, Jm, ct, hz);
        if (!(Jm[2][2] > 0.0) || !isfinite(Jm[2][2] + Jm[0][2] + Jm[1][2])) fl |= ORC_F_MAP;
        double* o = out + (size_t)r * 6;
        for (int I = 0; I < 3; ++I) {
            double v = 0.0;
            for (int K = 0; K < 3; ++K) v += Jm[I][K] * gh[K];
            o[I] = v;
            o[3 + I] = gh[I];
        }
        if (dim == 2) o[1] = 0.0;
        if (fl)
            for (int a = 0; a < 6; ++a) o[a] = NAN;
        if (flags) flags[r] = (uint8_t)fl;
    }
    return 0;
}

/* ------------------------------------------------------------------ volume smoothing (Sec. 3.6) */

/* Smoothed Jacobian determinant Jbar^N from Jbar^(N-1) (Sec. 3.6, Eq. VCT_bar_a).
 *
 * With the representative volume V_i = J_i / Jbar_i V, a neighbour pair (i, j)
 * exchanges the volume dV_ij = dJ_ij V,
 *   dJ_ij = C_V (r_e - |r^_ij|) / r_e (J_j / Jbar_j - J_i / Jbar_i),
 * and the two smoothed determinants become
 *   Jbar_i <- J_i Jbar_i / (J_i + Jbar_i dJ_ij),
 *   Jbar_j <- J_j Jbar_j / (J_j - Jbar_j dJ_ij).
 * The paper applies this to the neighbours j of a target particle i one after
 * the other, each update seen by the next.  Readings: every particle is a
 * target once, so each neighbour pair is visited from both of its ends; the
 * paper leaves the order of the targets open, so it is an argument (`order`,
 * a permutation of 0..n-1, NULL for index order), and the neighbours of a
 * target are taken in the order of its CSR row.  |r^_ij| is the projected
 * distance (r_e is the support radius of the neighbour set).  Sequential,
 * single-threaded.  jbar is updated in place. */
int orc_jbar_smooth(int dim, int64_t n, const double* pos, const double* J, double* jbar, double cv, double re,
                    const int64_t* order, const int64_t* row_ptr, const int32_t* col)
{
    if (dim != 2 && dim != 3) return -1;
    for (int64_t s = 0; s < n; ++s) {
        int64_t i = order ? order[s] : s;
        if (i < 0 || i >= n) return -1;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int64_t j = col[k];
            double r2 = 0.0;
            for (int a = 0; a < dim; ++a) {
                double d = pos[a * n + j] - pos[a * n + i];
                r2 += d * d;
            }
            double dJ = cv * (re - sqrt(r2)) / re * (J[j] / jbar[j] - J[i] / jbar[i]);
            double bi = J[i] * jbar[i] / (J[i] + jbar[i] * dJ);
            double bj = J[j] * jbar[j] / (J[j] - jbar[j] * dJ);
            jbar[i] = bi;
            jbar[j] = bj;
        }
    }
    return 0;
}

/* ------------------------------------------------ bathymetry adjoint, reading R2 */

/* Under reading R2 the particles' PHYSICAL positions are held fixed while the
 * bathymetry coefficients change, so the projected heights move with them,
 * z^_j = alpha(x_j, y_j) (z_j + beta(x_j, y_j)) (Sec. 2.1, Eq. VCT), and the
 * SPH(2) derivatives of every row change through the offsets r^_ij, the
 * correction matrices L_i and the moment matrices M_i (Eq. sec_SPH2).  The
 * oracle differentiates the literal two-stage formula by the complex step:
 * the rows below repeat the steps of orc_particle_geometry and
 * orc_particle_field in complex arithmetic (analytic in the heights; pivots and
 * kernel branches are chosen on real parts, which equal the real evaluation).
 * Field values, volumes, the loss target and the neighbour lists are fixed. */

/* -w'(r)/r of the normalised kernel at complex r^2 (r = csqrt(d2)) */
static double complex orc_c_gfac(int kernel, int dim, double R, double complex d2)
{
    double complex r = csqrt(d2);
    if (kernel == ORC_K_WENDLAND) {
        double C = (dim == 2) ? 7.0 / (M_PI * R * R) : 21.0 / (2.0 * M_PI * R * R * R);
        double complex q = r / R;
        if (creal(q) >= 1.0) return 0.0;
        double complex a = 1.0 - q;
        return C * 20.0 * a * a * a / (R * R);   /* -dw/dr / r with dw/dr = -20 C q a^3 / R */
    }
    double l = 0.5 * R;
    double ad = (dim == 2) ? 10.0 / (7.0 * M_PI * l * l) : 1.0 / (M_PI * l * l * l);
    double complex s = r / l;
    if (creal(s) <= 1.0) return ad * (3.0 - 2.25 * s) / (l * l);
    if (creal(s) < 2.0) {
        double complex t = 2.0 - s;
        return ad * 0.75 * t * t / (s * l * l);
    }
    return 0.0;
}

/* A X = B, complex, partial pivoting on the real parts; 1 if a pivot is 0 */
static int orc_cgepp(int n, double complex* A, int nrhs, double complex* B)
{
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(creal(A[r * n + c])) > fabs(creal(A[piv * n + c]))) piv = r;
        if (creal(A[piv * n + c]) == 0.0) return 1;
        if (piv != c) {
            for (int k = 0; k < n; ++k) { double complex t = A[c * n + k]; A[c * n + k] = A[piv * n + k]; A[piv * n + k] = t; }
            for (int k = 0; k < nrhs; ++k) { double complex t = B[c * nrhs + k]; B[c * nrhs + k] = B[piv * nrhs + k]; B[piv * nrhs + k] = t; }
        }
        for (int r = c + 1; r < n; ++r) {
            double complex f = A[r * n + c] / A[c * n + c];
            for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
            for (int k = 0; k < nrhs; ++k) B[r * nrhs + k] -= f * B[c * nrhs + k];
        }
    }
    for (int c = n - 1; c >= 0; --c)
        for (int k = 0; k < nrhs; ++k) {
            double complex s = B[c * nrhs + k];
            for (int j = c + 1; j < n; ++j) s -= A[c * n + j] * B[j * nrhs + k];
            B[c * nrhs + k] = s / A[c * n + c];
        }
    return 0;
}

/* The projected derivative vector D^ = [dz^, xx, yy, zz, xz, yz] of one field
 * at particle i by the two-stage formula of Eq. sec_SPH2 (second-order
 * gradient), in complex arithmetic.  The vertical projected coordinate of
 * particle j is zc[j] when zc is given, else the real one plus dzk at j == kp.
 * Returns 1 when a system is singular. */
static int orc_c_row_dhat(const orc_ctx* c, const double complex* zc, int64_t kp, double complex dzk, int64_t i,
                          const int32_t* nb, int64_t deg, const double* phi, double complex Dh[6])
{
    const int d = c->dim, m = c->m;
    const int64_t n = c->n;
    #define ZOF(j) (zc ? zc[j] : c->pos[(d - 1) * n + (j)] + ((j) == kp ? dzk : 0.0))
    double complex* r = malloc((size_t)(deg > 0 ? deg : 1) * 3 * sizeof(double complex));
    double complex* gt = malloc((size_t)(deg > 0 ? deg : 1) * 3 * sizeof(double complex));
    double complex* q = malloc((size_t)(deg > 0 ? deg : 1) * 6 * sizeof(double complex));
    double complex* F = malloc((size_t)(deg > 0 ? deg : 1) * sizeof(double complex));
    double complex* G = malloc((size_t)(deg > 0 ? deg : 1) * sizeof(double complex));
    int bad = !(r && gt && q && F && G);
    if (!bad) {
        double complex zi = ZOF(i);
        /* offsets, -w'(r)/r, monomials */
        double complex A[9] = {0}, L[9] = {0};
        for (int64_t k = 0; k < deg; ++k) {
            int64_t j = nb[k];
            double complex d2 = 0.0;
            for (int a = 0; a < d - 1; ++a) {
                r[3 * k + a] = c->pos[a * n + j] - c->pos[a * n + i];
                d2 += r[3 * k + a] * r[3 * k + a];
            }
            r[3 * k + d - 1] = ZOF(j) - zi;
            d2 += r[3 * k + d - 1] * r[3 * k + d - 1];
            F[k] = d2;
            G[k] = orc_c_gfac(c->kernel, d, c->R, d2);
            double complex* rq = r + 3 * k;
            double complex* qq = q + 6 * k;
            if (d == 2) { qq[0] = rq[0] * rq[0]; qq[1] = rq[1] * rq[1]; qq[2] = rq[0] * rq[1]; }
            else {
                qq[0] = rq[0] * rq[0]; qq[1] = rq[1] * rq[1]; qq[2] = rq[2] * rq[2];
                qq[3] = rq[0] * rq[1]; qq[4] = rq[0] * rq[2]; qq[5] = rq[1] * rq[2];
            }
            /* A_i = sum_j V_j grad w_ij (x) r_ij, grad w_ij = G r_ij */
            double V = c->vol[j];
            for (int a = 0; a < d; ++a)
                for (int b = 0; b < d; ++b) A[a * d + b] += V * G[k] * rq[a] * rq[b];
        }
        for (int a = 0; a < d; ++a) L[a * d + a] = 1.0;
        bad = orc_cgepp(d, A, d, L);
        /* corrected gradients L grad w, Q_i, F_ij, p_ij, M_i */
        double complex Q[18] = {0}, M[36] = {0}, b[6] = {0}, g1[3] = {0};
        if (!bad) {
            for (int64_t k = 0; k < deg; ++k)
                for (int a = 0; a < d; ++a) {
                    double complex t = 0.0;
                    for (int bb = 0; bb < d; ++bb) t += L[a * d + bb] * G[k] * r[3 * k + bb];
                    gt[3 * k + a] = t;
                }
            for (int64_t k = 0; k < deg; ++k) {
                double V = c->vol[nb[k]];
                for (int mm = 0; mm < m; ++mm)
                    for (int a = 0; a < d; ++a) Q[mm * d + a] += V * q[6 * k + mm] * gt[3 * k + a];
                double pij = phi[nb[k]] - phi[i];
                for (int a = 0; a < d; ++a) g1[a] += V * pij * gt[3 * k + a];
            }
            for (int64_t k = 0; k < deg; ++k) {
                double complex rg = 0.0;
                for (int a = 0; a < d; ++a) rg += r[3 * k + a] * gt[3 * k + a];
                double complex d2 = F[k];
                F[k] = rg / (d2 * d2);
                double complex p[6];
                for (int mm = 0; mm < m; ++mm) {
                    double complex t = 0.0;
                    for (int a = 0; a < d; ++a) t += Q[mm * d + a] * r[3 * k + a];
                    p[mm] = q[6 * k + mm] - t;
                }
                double V = c->vol[nb[k]];
                double complex rg1 = 0.0;
                for (int a = 0; a < d; ++a) rg1 += r[3 * k + a] * g1[a];
                double complex t = V * F[k] * ((phi[nb[k]] - phi[i]) - rg1);
                for (int aa = 0; aa < m; ++aa) {
                    b[aa] += t * q[6 * k + aa];
                    for (int bb = 0; bb < m; ++bb) M[aa * m + bb] += V * F[k] * q[6 * k + aa] * p[bb];
                }
            }
            bad = orc_cgepp(m, M, 1, b);
        }
        if (!bad) {
            double complex D[6];
            for (int mm = 0; mm < m; ++mm) D[mm] = 2.0 * b[mm];
            double complex g2[3];
            for (int a = 0; a < d; ++a) {
                double complex t = 0.0;
                for (int mm = 0; mm < m; ++mm) t += Q[mm * d + a] * D[mm];
                g2[a] = g1[a] - 0.5 * t;
            }
            if (d == 2) {
                Dh[0] = g2[1]; Dh[1] = D[0]; Dh[2] = 0.0; Dh[3] = D[1]; Dh[4] = 0.5 * D[2]; Dh[5] = 0.0;
            } else {
                Dh[0] = g2[2]; Dh[1] = D[0]; Dh[2] = D[1]; Dh[3] = D[2]; Dh[4] = 0.5 * D[4]; Dh[5] = 0.5 * D[5];
            }
        }
    }
    #undef ZOF
    free(r); free(gt); free(q); free(F); free(G);
    return bad ? 1 : 0;
}

/* d loss / d z^_k at sampled particles k, loss = sum_i (lap_i - g_i)^2 with
 * lap_i = c_trans_i . D^_i, for a fixed mapping: by the complex step of z^_k
 * alone, which changes the rows of k and of its neighbours.  u_i = 2 (lap_i -
 * g_i) comes from the real evaluation.  With ct_dep = 0 c_trans is held at
 * its value (only the SPH(2) derivatives move). */
int orc_r2_dzhat(int dim, int64_t n, const double* pos, const double* vol, const double* phi, int kernel, double R,
                 int map_kind, double Hhat, double H, double dmin, double eps, int nterms, const double* terms,
                 const double* u, int ct_dep, int64_t nk, const int64_t* ks, const int64_t* row_ptr,
                 const int32_t* col, double* out)
{
    orc_ctx c;
    ctx_init(&c, dim, n, pos, vol, kernel, R, map_kind, Hhat, H, dmin, eps, nterms, terms, 2);
    const double h = 1e-30;
    int status = 0;
    #pragma omp parallel for schedule(dynamic, 4) reduction(| : status)
    for (int64_t s = 0; s < nk; ++s) {
        int64_t k = ks ? ks[s] : s;
        const double complex dz = h * _Complex_I;
        double acc = 0.0;
        for (int64_t e = row_ptr[k] - 1; e < row_ptr[k + 1]; ++e) {
            int64_t i = e < row_ptr[k] ? k : col[e];   /* the row of k first, then its neighbours' */
            double complex Dh[6];
            if (orc_c_row_dhat(&c, NULL, k, dz, i, col + row_ptr[i], row_ptr[i + 1] - row_ptr[i], phi, Dh)) {
                status = 1;
                continue;
            }
            double x = pos[i], y = (dim == 3) ? pos[n + i] : 0.0, zh = pos[(dim - 1) * n + i];
            double complex ct[6];
            orc_c_map_ct(&c.map, dim, x, y, (ct_dep && i == k) ? zh + dz : zh, i, -1, 0.0, ct);
            double complex lap = 0.0;
            for (int q = 0; q < 6; ++q) lap += ct[q] * Dh[q];
            acc += u[i] * cimag(lap) / h;
        }
        out[s] = acc;
    }
    return status ? -1 : 0;
}

/* Projected positions of physical points (x, [y], z): z^ = alpha (z + beta). */
int orc_project(int dim, int64_t n, const double* phys, int map_kind, double Hhat, double H, double dmin, double eps,
                int nterms, const double* terms, double* proj)
{
    orc_map mp;
    mp.kind = map_kind; mp.Hhat = Hhat; mp.H = H; mp.dmin = dmin; mp.eps = eps;
    mp.nterms = nterms; mp.terms = terms;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double x = phys[i], y = (dim == 3) ? phys[n + i] : 0.0, z = phys[(dim - 1) * n + i];
        double ab[12];
        orc_r_alpha_beta(&mp, dim, x, y, i, -1, 0.0, ab);
        for (int a = 0; a < dim - 1; ++a) proj[a * n + i] = phys[a * n + i];
        proj[(dim - 1) * n + i] = ab[0] * (z + ab[6]);
    }
    return 0;
}

/* d loss / d coef_t under reading R2, by the complex step of coef_t through
 * the whole evaluation: every particle's projected height
 * z^_j = alpha_c (z_j + beta_c) with the perturbed mapping, every row's D^ and
 * c_trans, then the loss.  phys: physical positions (x, [y], z); the
 * neighbour lists are those of the real projected positions. */
int orc_r2_dtheta(int dim, int64_t n, const double* phys, const double* vol, const double* phi, const double* g,
                  int kernel, double R, int map_kind, double Hhat, double H, double dmin, double eps, int nterms,
                  const double* terms, int nt, const int32_t* tlist, const int64_t* row_ptr, const int32_t* col,
                  double* dtheta)
{
    orc_map mp;
    mp.kind = map_kind; mp.Hhat = Hhat; mp.H = H; mp.dmin = dmin; mp.eps = eps;
    mp.nterms = nterms; mp.terms = terms;
    const double h = 1e-30;
    double* proj = malloc((size_t)(n > 0 ? n : 1) * dim * sizeof(double));
    double complex* zc = malloc((size_t)(n > 0 ? n : 1) * sizeof(double complex));
    double* part = malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!proj || !zc || !part) { free(proj); free(zc); free(part); return -1; }
    orc_project(dim, n, phys, map_kind, Hhat, H, dmin, eps, nterms, terms, proj);
    orc_ctx c;
    ctx_init(&c, dim, n, proj, vol, kernel, R, map_kind, Hhat, H, dmin, eps, nterms, terms, 2);
    int status = 0;
    for (int tt = 0; tt < nt; ++tt) {
        const int t = tlist[tt];
        const double complex dc = h * _Complex_I;
        #pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < n; ++j) {
            double x = phys[j], y = (dim == 3) ? phys[n + j] : 0.0, z = phys[(dim - 1) * n + j];
            double complex ab[12];
            orc_c_alpha_beta(&mp, dim, x, y, j, t, dc, ab);
            zc[j] = ab[0] * (z + ab[6]);
        }
        #pragma omp parallel for schedule(dynamic, 16) reduction(| : status)
        for (int64_t i = 0; i < n; ++i) {
            double complex Dh[6];
            part[i] = 0.0;
            if (orc_c_row_dhat(&c, zc, -1, 0.0, i, col + row_ptr[i], row_ptr[i + 1] - row_ptr[i], phi, Dh)) {
                status = 1;
                continue;
            }
            double x = phys[i], y = (dim == 3) ? phys[n + i] : 0.0;
            double complex ct[6];
            orc_c_map_ct(&mp, dim, x, y, zc[i], i, t, dc, ct);
            double complex lap = 0.0;
            for (int q = 0; q < 6; ++q) lap += ct[q] * Dh[q];
            double complex e = lap - g[i];
            part[i] = cimag(e * e) / h;
        }
        double sum = 0.0, comp = 0.0;   /* fixed order, Kahan */
        for (int64_t i = 0; i < n; ++i) {
            double yv = part[i] - comp, tv = sum + yv;
            comp = (tv - sum) - yv;
            sum = tv;
        }
        dtheta[tt] = sum;
    }
    free(proj); free(zc); free(part);
    return status ? -1 : 0;
}
