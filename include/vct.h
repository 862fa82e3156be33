/* vct.h -- C ABI of the VCT-SPH(2) operator library for AMD MI355X (gfx950).
 *
 * The library evaluates second-order-accurate SPH derivative operators
 * (gradient, Laplacian, cross derivatives) of particle fields, computed in the
 * projected space of a vertical coordinate transformation (VCT) and mapped back
 * to physical space:
 *   - VCT:  x^ = x, y^ = y, z^ = alpha(x,y) (z + beta(x,y))        paper Sec. 2.1, Eq. VCT
 *   - gradient  grad phi = J grad^ phi                              Eq. grad_VCT
 *   - Laplacian lap phi = c_trans . D^ phi                          Eq. lap_VCT
 *   - alpha/beta for E-, BF-, BFE- and sigma-SPH                     Sec. 2.2
 *   - neighbour set S_i = { j != i : |r^_ij| < R }                   Sec. 3.1, Eq. SPH_neighbor_set
 *   - first-order corrected gradient (L_i)                          Sec. 3.1, Eq. gra_1st
 *   - SPH(2) second derivatives (M_i, F_ij, p_ij, q_ij)             Sec. 3.1, Eq. sec_SPH2
 *
 * Conventions for every entry point
 *   - Pointers are DEVICE pointers unless marked (host).  The library never
 *     allocates device memory: the caller owns inputs, outputs and scratch
 *     ("workspace", sized by the matching *_workspace_size query).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls are stream-ordered and asynchronous unless marked SYNC, in which
 *     case they wait for their own work on `stream` before returning.
 *   - Per-particle arrays are in the cell-sorted order produced by
 *     vct_build_cells unless stated otherwise; perm maps sorted -> original.
 *   - Layouts: positions SoA [dim][n] (2-D sets use the vertical plane (x, z));
 *     fields [nf][n]; outputs [nf][n][n_out]; state SoA [stride][n];
 *     neighbour lists in CSR form (vct_nlist).
 *   - Return value: VCT_OK (0); a positive warning (outputs written); or a
 *     negative error, in which case nothing was launched unless stated.
 *     Argument errors are detected on the host before any HIP call.  Nothing
 *     aborts or throws across the ABI.  Calls that share a workspace or outputs
 *     must not overlap.
 */
#ifndef VCT_H
#define VCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
    VCT_OK = 0,
    VCT_W_FLAGGED = 1,      /* some particles were flagged; their outputs are NaN */
    VCT_W_NOCONV = 2,       /* an iterative solve stopped before its tolerance (result written) */
    VCT_E_ARG = -1,         /* invalid argument (null pointer, size, enum, range) */
    VCT_E_HIP = -2,         /* a HIP runtime call or kernel launch failed */
    VCT_E_CAPACITY = -3,    /* an output array is too small; the required size is reported */
    VCT_E_NONFINITE = -4,   /* a non-finite input position */
    VCT_E_WORKSPACE = -5,   /* workspace missing or smaller than the size query returns */
    VCT_E_WINDOW = -6       /* a chunk's neighbour window exceeds 65535 particles (16-bit offsets) */
};

/* ---------------------------------------------------------------- enums */
enum { VCT_KERNEL_WENDLAND_C2 = 0, VCT_KERNEL_CUBIC_SPLINE = 1 };

/* arithmetic of vct_apply_ops */
enum {
    VCT_FP64 = 0,           /* FP64 pair terms and sums, FP64 state */
    VCT_MIXED = 1,          /* FP32 pair terms and FP32 sums, FP32 copy of the FP64-solved state */
    VCT_MIXED_S64 = 2       /* FP32 pair terms and FP32 sums, FP64 state */
};

/* mapping kinds (paper Sec. 2.2) */
enum { VCT_MAP_IDENTITY = 0, VCT_MAP_E = 1, VCT_MAP_BF = 2, VCT_MAP_BFE = 3, VCT_MAP_SIGMA = 4,
       VCT_MAP_PER_PARTICLE = 5 };

/* one separable factor B(s) of a bathymetry term */
enum { VCT_BASIS_ONE = 0, VCT_BASIS_LIN = 1, VCT_BASIS_COS = 2, VCT_BASIS_SIN = 3 };

#define VCT_MAX_TERMS 32

/* Output selection.  Rows of one particle's output record are the selected
 * groups concatenated in this bit order:
 *   GRAD   physical gradient            2-D: x, z         3-D: x, y, z
 *   LAP    physical Laplacian           1
 *   CROSS  physical cross derivatives   2-D: xz           3-D: xy, xz, yz
 *   HESS   physical Hessian             2-D: xx, zz, xz   3-D: xx, yy, zz, xy, xz, yz
 *   PGRAD  projected gradient           2-D: x^, z^       3-D: x^, y^, z^
 *   PHESS  projected second derivatives (same component order as HESS)
 *   PZ     the projected derivatives whose coefficients in the physical
 *          Laplacian depend on the mapping (Eq. lap_VCT)
 *                                       2-D: z^, z^z^, x^z^
 *                                       3-D: z^, z^z^, x^z^, y^z^
 *          (the same values as those rows of PGRAD and PHESS; enough, with
 *          LAP, for the adjoint's dtheta, at less than half their state)
 * VCT_OPT_GRAD1 makes every gradient (and the dz^ entering LAP, CROSS and HESS)
 * the first-order corrected one (Eq. gra_1st) instead of the second-order
 * gradient SPH(2) provides.                                                    */
enum {
    VCT_OUT_GRAD = 1u << 0,
    VCT_OUT_LAP = 1u << 1,
    VCT_OUT_CROSS = 1u << 2,
    VCT_OUT_HESS = 1u << 3,
    VCT_OUT_PGRAD = 1u << 4,
    VCT_OUT_PHESS = 1u << 5,
    VCT_OUT_PZ = 1u << 6,
    VCT_OPT_GRAD1 = 1u << 8
};
#define VCT_OUT_DEFAULT (VCT_OUT_GRAD | VCT_OUT_LAP | VCT_OUT_CROSS)

/* per-particle flag bits written by vct_moments */
enum {
    VCT_FLAG_FEW = 1,        /* fewer than d + m neighbours (d + m = 5 in 2-D, 9 in 3-D) */
    VCT_FLAG_SINGULAR_A = 2, /* first-order correction matrix numerically singular */
    VCT_FLAG_SINGULAR_M = 4, /* SPH(2) moment matrix numerically singular */
    VCT_FLAG_NONFINITE = 8,  /* non-finite position or volume at the particle or a neighbour */
    VCT_FLAG_DUPLICATE = 16, /* a neighbour at zero distance */
    VCT_FLAG_MAP = 32        /* the mapping is invalid at the particle: alpha (or one of the
                                mapping coefficients) not finite, or alpha <= 0 (Sec. 2.1
                                requires alpha > 0; e.g. a dry sigma column without limiter) */
};

/* Bottom elevation term: h(x, y) += coef * Bx(x) * By(y) with
 * B = 1, s, cos(2 pi f s) or sin(2 pi f s) (basis kind, frequency f).
 * In 2-D only the x factor varies (By is evaluated at y = 0, derivatives 0). */
typedef struct {
    double coef;
    int32_t bx, by;
    double fx, fy;
} vct_term;

/* Vertical coordinate transformation (paper Sec. 2.2):
 *   IDENTITY  alpha = 1,            beta = 0
 *   E         alpha = Hhat / H,     beta = 0
 *   BF        alpha = 1,            beta = -h
 *   BFE       alpha = Hhat / H,     beta = -h
 *   SIGMA     alpha = Hhat / D_eff, beta = D_eff - H,  D = H - h,
 *             D_eff = (D + dmin + sqrt((D - dmin)^2 + eps^2)) / 2 when dmin > 0 or
 *             eps > 0 (the paper asks for a constant alpha outside an unstated
 *             applicable range; this smooth limiter is the reading used), else D.
 *             dmin > 0 needs eps > 0 (VCT_E_ARG otherwise: with eps = 0 the
 *             limiter is a hard max whose second derivative is undefined at
 *             D = dmin).  Particles where alpha is not positive and finite are
 *             flagged VCT_FLAG_MAP by vct_moments.
 *   PER_PARTICLE  alpha, beta and their first and second horizontal
 *             derivatives given at every point (a measured or tabulated
 *             bottom, any transformation of the form of Eq. VCT): `coef` is a
 *             DEVICE array [12][coef_n] with rows alpha, alpha_x, alpha_y,
 *             alpha_xx, alpha_xy, alpha_yy, beta, beta_x, beta_y, beta_xx,
 *             beta_xy, beta_yy, in the order of the call's points (sorted
 *             order for the calls on a neighbour list); coef_n must equal the
 *             call's number of points and nterms must be 0 (no bathymetry
 *             coefficients to differentiate: the adjoints give no dtheta, and
 *             vct_apply_ops_adjoint_r2 returns VCT_E_ARG).  In 2-D the y
 *             rows are ignored.  Read by the device during the call.
 * `terms` is a HOST pointer to nterms (<= VCT_MAX_TERMS) entries; it is read
 * during the call only.                                                        */
typedef struct {
    int32_t kind;
    int32_t nterms;
    double Hhat, H, dmin, eps;
    const vct_term* terms;
    const double* coef;     /* PER_PARTICLE only, else NULL */
    int64_t coef_n;
} vct_map;

/* ---------------------------------------------------------------- queries */

/* Status name (static string; never NULL). */
const char* vct_status_string(int status);

/* Text of the last HIP error seen by this thread (static storage). */
const char* vct_last_error(void);

/* Background-cell grid over the projected box [lo, hi) for support radius R:
 * per axis nc = max(1, floor((hi - lo) / (R (1 + 2^-20)))) cells of size
 * (hi - lo) / nc >= R.  Positions outside the box are clamped to the boundary
 * cells, which keeps the search correct (clamping never separates two points
 * closer than one cell).  Writes dims (host, 3 entries; unused axes = 1) and
 * returns the number of cells, or a negative status.  Host only.              */
int64_t vct_grid_dims(int dim, const double* lo, const double* hi, double R, int64_t* dims);

/* Rows of one particle's output record for `out_mask` (0 if invalid). */
int vct_n_out(int dim, uint32_t out_mask);

/* Values per particle in the state written by vct_moments:
 * nL + n_out * (d + m) + n_out * d, nL = 3 (2-D) or 6 (3-D).  0 if invalid. */
int vct_state_stride(int dim, uint32_t out_mask);

/* ---------------------------------------------------------------- launch timing */

/* Per-kernel launch timing, for measurement.  While enabled, every kernel
 * launch made by this library is bracketed by two HIP events recorded on the
 * stream the kernel is launched on.  vct_timing_count and vct_timing_get wait
 * for the recorded events (SYNC on them) and fold them, per kernel name, into
 * a launch count and a summed duration in milliseconds.  Off by default; when
 * off a launch pays one atomic load.  Do not enable while a stream of this
 * library is being captured into a graph.  Host only, thread-safe.
 * vct_timing_enable returns the previous state (0/1); disabling folds the
 * pending records.  vct_timing_reset drops all records and totals.            */
int vct_timing_enable(int on);
void vct_timing_reset(void);
/* Number of kernel names with folded records. */
int vct_timing_count(void);
/* Entry idx < vct_timing_count(): kernel name (static string owned by the
 * library), launches and summed milliseconds (host pointers).  VCT_E_ARG for
 * a bad index or a NULL pointer.                                              */
int vct_timing_get(int idx, const char** name, int64_t* launches, double* total_ms);

/* ---------------------------------------------------------------- device checks */

/* A debug build of the library (compiled with VCT_DEVICE_CHECKS=1) checks on
 * the device the indices its kernels derive from the neighbour data: window
 * offsets against their window (col16 of every entry point that reads it),
 * the neighbour search's staged hit words and expanded rows against their
 * buffers, and the push form's
 * accumulator indices against the column window.  A failed check sets its bit
 * (below) and the index is replaced by 0, which stays in bounds, so every
 * kernel still runs to its end; the outputs are then meaningless.
 * vct_device_checks waits for the device (SYNC), ORs the bits set since the
 * previous call into *bits and clears them.  Returns 1 for a checked build, 0
 * for a release build (*bits = 0: nothing is checked), or a negative status.
 * Not meant for concurrent use with running work.  Host only.                 */
enum {
    VCT_CHECK_WINDOW = 1,     /* a window offset at or past the end of its window */
    VCT_CHECK_CAPACITY = 2,   /* an index past the buffer a count is staged in */
    VCT_CHECK_ACCUM = 4       /* an accumulator index past the column window */
};
int vct_device_checks(uint32_t* bits);

/* ---------------------------------------------------------------- cells */

size_t vct_build_cells_workspace_size(int dim, int64_t n, int64_t ncell);

/* Background-cell sort (paper Sec. 3.4 performs neighbour searches with
 * background cells).  Buckets the n particles (positions `pos`, SoA [dim][n],
 * ORIGINAL order, projected space) into the grid of vct_grid_dims and sorts
 * them by (cell, original index): cells in lexicographic order of (x, y, z)
 * cell coordinates with z fastest.
 *   perm       [n]          sorted index -> original index
 *   pos_sorted [dim][n]     positions in sorted order
 *   cell_start [ncell + 1]  first sorted index of every cell; cell c holds
 *                           [cell_start[c], cell_start[c+1])
 * SYNC.  Returns VCT_E_NONFINITE (outputs undefined) if any coordinate is not
 * finite.  n == 0 is valid (cell_start is zero-filled).                        */
int vct_build_cells(int dim, int64_t n, const double* pos, const double* lo, const double* hi,
                    double R, int32_t* perm, double* pos_sorted, int64_t* cell_start,
                    int64_t ncell, void* ws, size_t ws_bytes, void* stream);

/* Gather per-particle arrays into sorted order: dst[c][s] = src[c][perm[s]] for
 * ncomp components of n values each.  vct_scatter_sorted is the inverse
 * (dst[c][perm[s]] = src[c][s]).                                               */
int vct_gather_sorted(int64_t n, int ncomp, const int32_t* perm, const double* src, double* dst,
                      void* stream);
int vct_scatter_sorted(int64_t n, int ncomp, const int32_t* perm, const double* src, double* dst,
                       void* stream);

/* ---------------------------------------------------------------- neighbours */

/* Neighbour structure of one cell-sorted particle set.  A host struct of
 * device pointers that the caller allocates; vct_neighbors fills the chunk
 * table, row_ptr and the columns.
 *
 * Chunks: the particles of each background-cell column ((x, y) column in 3-D,
 * x column in 2-D) are split into runs of at most 64 consecutive sorted
 * particles.  A chunk's window is the concatenation, in increasing order, of
 * the sorted-index ranges of the 3^(d-1) columns around its own, restricted
 * to the z cells the chunk spans plus one on each side; every neighbour of a
 * chunk's particles lies in it.  Kernels stage the window in LDS.
 *
 * Columns of row i are ascending; `col` holds sorted particle indices and
 * `col16` the same neighbours as offsets into the window of i's chunk.  At
 * least one of them must be given to vct_neighbors; vct_moments,
 * vct_apply_ops and vct_apply_ops_adjoint read col16, which must be 16-byte
 * aligned (VCT_E_ARG otherwise).                                             */
typedef struct {
    int32_t dim;            /* 2 or 3 */
    int32_t reserved;
    int64_t n;              /* particles */
    int64_t ncell;          /* cells (vct_grid_dims) */
    int64_t chunk_cap;      /* capacity of the chunk arrays, >= vct_chunk_capacity() */
    double lo[3], hi[3];    /* projected box given to vct_build_cells (unused entries ignored) */
    double R;               /* support radius */
    const int64_t* cell_start;  /* [ncell + 1], from vct_build_cells */
    int64_t* chunk_off;     /* [ncols + 1]: first chunk of every column; chunk_off[ncols] = chunks */
    int32_t* chunk_start;   /* [chunk_cap + 1]: first sorted particle of every chunk */
    int32_t* chunk_info;    /* [chunk_cap][4]: column, first z cell, last z cell, 0 */
    int64_t* row_ptr;       /* [n + 1] */
    int32_t* col;           /* [nnz] or NULL */
    uint16_t* col16;        /* [nnz] or NULL; 16-byte aligned */
    int32_t* col_t;         /* [nnz] or NULL: for entry e = (i, j) of row i, the position of
                               the entry (j, i) in row j (needs col); read by the adjoint */
    int64_t nnz;            /* written by vct_neighbors (the total of row_ptr) */
    int32_t* chunk_win;     /* [chunk_cap][32] or NULL: every chunk's window (its column
                               ranges), written by vct_neighbors and read by the other
                               calls instead of recomputing it from cell_start */
} vct_nlist;

/* Entries needed in the chunk arrays of a set of n particles on ncell cells. */
int64_t vct_chunk_capacity(int dim, int64_t n, int64_t ncell);

/* Workspace of vct_neighbors: counts, scan tiles, flags and a staging area of
 * 128 16-bit entries per particle (256 n bytes). */
size_t vct_neighbors_workspace_size(int64_t n, int64_t ncell);

/* Neighbour lists S_i = { j != i : d2(i,j) < R*R } (Eq. SPH_neighbor_set) of
 * the cell-sorted particles pos_sorted (SoA [dim][n]).  d2 is defined in FP64
 * as ((dx*dx + dy*dy) + dz*dz) with dx = x_j - x_i and no fused multiply-add,
 * so lists are reproducible bit for bit (a conservative FP32 pre-test decides
 * the clear cases; the rest use that exact FP64 expression).
 * Protocol: the chunk table and row_ptr are always written and *nnz_out (host)
 * and nl->nnz receive the total.  If both col and col16 are NULL the call
 * stops there (VCT_OK).  If col_cap < nnz it returns VCT_E_CAPACITY (row_ptr
 * and nnz are still valid, so the caller can size the columns and call again).
 * Otherwise the columns are written (ascending within a row), and col_t when
 * it is given (it needs col; the neighbour relation is symmetric, so every
 * entry has its transpose).  With columns requested and reuse_row_ptr == 0 the
 * search runs once: the hits of every chunk's candidate window are staged in
 * the workspace as bit words while the rows are counted, then expanded into
 * the rows behind row_ptr; when some chunk's window is wider than 2048
 * particles (more words than its share of the workspace holds) the search is
 * repeated to write the columns in place.  With reuse_row_ptr != 0
 * the chunk table and row_ptr are not recomputed (they must hold the result of
 * an earlier call on the same inputs) and the search writes the columns in
 * place.  Returns VCT_E_WINDOW if some window exceeds 65535 particles (col16
 * cannot address it).  SYNC (reads nnz).                                       */
int vct_neighbors(vct_nlist* nl, const double* pos_sorted, int64_t col_cap, int64_t* nnz_out, int reuse_row_ptr,
                  void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- moments */

/* Per-particle moment assembly and solve, always in FP64 (Eqs. gra_1st and
 * sec_SPH2).  For every particle i it forms the first-order correction matrix
 * and the SPH(2) system, equivalently the (d+m) x (d+m) block system of the
 * Taylor moments (m = 3 in 2-D, 6 in 3-D), eliminates the first block row
 * (Schur complement M), inverts M by Gauss-Jordan elimination with partial
 * pivoting, and folds the solution with the VCT coefficients of `map` at the particle into
 * the state consumed by vct_apply_ops:
 *   state[k][i], k < nL               dimensionless first-order correction
 *                                     matrix (symmetric, upper triangle) in
 *                                     units of R
 *   state[nL + o*(d+m) + c][i]         coefficient of neighbour sum c in output
 *                                     row o of `out_mask`
 *   state[nL + n_out*(d+m) + o*d + a][i]  response of output row o to a unit
 *                                     projected gradient along axis a (the
 *                                     operator applied to a linear field)
 * state64 [stride][n] (FP64) and state32 (its FP32 rounding, same layout)
 * are each optional, but one of them must be given: a caller that only runs
 * the mixed apply can skip the FP64 copy.  flags [n] (may be NULL) receives VCT_FLAG_* bits; flagged particles
 * get NaN state rows, hence NaN outputs.  If n_flagged (host) is not NULL the
 * call is SYNC and returns VCT_W_FLAGGED when the count is non-zero.          */
int vct_moments(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                const vct_map* map /* host */, uint32_t out_mask, double* state64, float* state32, uint8_t* flags,
                int64_t* n_flagged, void* ws, size_t ws_bytes, void* stream);

size_t vct_moments_workspace_size(int dim, int64_t n);

/* vct_moments with a second state from the same solve (Eqs. gra_1st and
 * sec_SPH2; Sec. 2.1 for the fold): the inverse of each particle's moment
 * system is folded twice, with out_mask into state64 / state32 and with
 * out_mask2 into state64_2 / state32_2 (layout of each as in vct_moments,
 * its stride from its own mask), so a caller that needs two row sets (the
 * FP32 state of a mixed forward and the FP64 LAP + PZ state of its adjoint,
 * say) reads the sums and inverts once.  The map, the flags and the
 * VCT_OPT_GRAD1 choice are shared: masks that differ in VCT_OPT_GRAD1 are
 * VCT_E_ARG.  With state64_2 and state32_2 both NULL this is vct_moments.
 * Each state is bitwise the one a vct_moments call with its mask writes.
 * Other arguments and errors as in vct_moments.                             */
int vct_moments_ex(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                   const vct_map* map /* host */, uint32_t out_mask, double* state64, float* state32,
                   uint32_t out_mask2, double* state64_2, float* state32_2, uint8_t* flags, int64_t* n_flagged,
                   void* ws, size_t ws_bytes, void* stream);

/* The solve and fold of vct_moments alone, from the moment sums that the last
 * vct_moments call left in `ws`.  The sums depend only on the neighbour list,
 * positions, volumes, kernel and R, not on `map` or `out_mask`, so a second
 * state for other outputs or another map (the LAP and PZ rows of an adjoint
 * after a forward that wrote the default outputs, say) costs one
 * solve instead of two sweeps over the rows.  `ws` must come from a
 * vct_moments call on the same nl, pos_sorted and vol_sorted, ordered before
 * this one on the stream, and must not be used by another call in between;
 * the library cannot check this.  Arguments, state layout, flags and
 * n_flagged as in vct_moments; the results are bitwise those of a vct_moments
 * call with the same map and out_mask.                                         */
int vct_moments_resolve(const vct_nlist* nl, const double* pos_sorted, const vct_map* map /* host */,
                        uint32_t out_mask, double* state64, float* state32, uint8_t* flags, int64_t* n_flagged,
                        void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- apply */

/* Apply the operators to nf fields (Eqs. grad_VCT, lap_VCT, sec_SPH2):
 *   a_i = sum_j V_j phi_ij grad w_ij,   s_i = sum_j V_j F_ij q_ij phi_ij
 * (phi_ij = phi_j - phi_i), then out_i = P_i [a_i; s_i] with the state of
 * vct_moments (same out_mask).  The sums are taken in two passes over the row:
 * the first gives the first-order gradient G_i = L_i a_i, the second sums the
 * residual psi_ij = phi_ij - r_ij . G_i (formed in FP64), and
 * out_i = P_i [a_i(psi); s_i(psi)] + W_i G_i.  This equals the one-pass result
 * exactly (the operator reproduces linear fields) while keeping the summed
 * terms second-order small, so rounding in the sums is not amplified by the
 * cancellation of the first-order parts.  `state` is FP64 for VCT_FP64 and
 * VCT_MIXED_S64, FP32 (state32) for VCT_MIXED.  phi_sorted [nf][n] FP64,
 * out [nf][n][n_out] FP64.  In the mixed forms r_ij, phi_ij and psi_ij are
 * formed in FP64 and rounded once to FP32; the pair terms and sums are FP32;
 * the final product with the state is FP32 and stored as FP64.                */
int vct_apply_ops(const vct_nlist* nl, int nf, const double* phi_sorted, const double* pos_sorted,
                  const double* vol_sorted, int kernel, const void* state, uint32_t out_mask, int precision,
                  double* out, void* stream);

/* vct_apply_ops with the first-order gradient of the first pass exposed
 * (Eq. gra_1st).  G~_i = L_i a_i is that gradient in projected coordinates and
 * in units of 1/R (the gradient times R).  g_out [nf][d][n] FP32 (device, may
 * be NULL) receives G~ as the call computed it, in any precision.  g_in
 * [nf][d][n] FP32 (device, may be NULL) is read by VCT_FP64 only: it replaces
 * the call's own first pass, which is then skipped (chunks whose neighbour
 * windows exceed the LDS staging still run theirs).  Because
 * out_i = P_i [a_i(psi); s_i(psi)] + W_i G_i holds for any G_i, a G~ from a
 * mixed call on the same fields, positions, volumes and neighbour list (the
 * FP32 rounding of the same gradient) gives the FP64 result up to rounding;
 * a G~ of anything else gives a wrong result that the library cannot detect.
 * The other precisions ignore g_in.  Passing both is VCT_E_ARG.  Other
 * arguments, layout and errors as in vct_apply_ops.                         */
int vct_apply_ops_ex(const vct_nlist* nl, int nf, const double* phi_sorted, const double* pos_sorted,
                     const double* vol_sorted, int kernel, const void* state, uint32_t out_mask, int precision,
                     double* out, float* g_out, const float* g_in, void* stream);

/* ---------------------------------------------------------------- adjoint */

size_t vct_adjoint_workspace_size(int dim, int64_t n, int64_t nnz, int nterms);

/* Adjoint of the physical Laplacian (not in the paper; built on Eqs. lap_VCT
 * and sec_SPH2).  With lap_i = sum_j W_ij phi_ij the linear operator of
 * vct_apply_ops (FP64), and u [n] the cotangent of lap:
 *   dphi_k   = sum_{i in S_k} u_i W_ik - u_k sum_{j in S_k} W_kj
 *   dtheta_t = sum_i u_i (d c_trans_i / d coef_t) . D^ phi_i
 *              for every bathymetry term t of `map` (projected positions held
 *              fixed).
 * dphi, two forms; each evaluates every weight W_ij once and gives the same
 * bits on every run (no floating-point atomics):
 *   with nl->col_t: every particle i writes u_i W_ij for its row into the
 *     workspace at the transposed position col_t[e], then every particle k sums
 *     its row of that buffer in row order (the map costs a binary search per
 *     entry to build, so this pays when one geometry serves many adjoints);
 *   without (push form; needs nl->chunk_win, VCT_E_ARG otherwise): per
 *     background-cell column, every particle i adds
 *     u_i W_ij (and -u_i sum_j W_ij to itself) to accumulators of the
 *     column's window held in LDS as exact integers: each term is scaled by
 *     2^k from a per-column bound M on the terms (k = 61 - ilogb(M)), rounded
 *     and summed in two 64-bit integer parts, so the order of arrival does not
 *     matter; the column's totals go to one of 3^(d-1) slots per particle,
 *     summed in slot order.  The rounding of each term is at most 2^-62 M.
 * dtheta: per particle from D^ phi_i, reduced in a fixed order.
 * `state64` must come from vct_moments (or vct_moments_resolve) with out_mask
 * containing VCT_OUT_LAP and either VCT_OUT_PZ or both VCT_OUT_PGRAD and
 * VCT_OUT_PHESS (pass the same mask).
 * `proj` [n][n_out] FP64 is the output of vct_apply_ops (nf = 1, VCT_FP64,
 * the same state and mask) for the field whose dtheta is wanted; it supplies
 * the projected derivatives that c_trans weights (dz^, z^z^, x^z^, y^z^) and
 * is needed only when dtheta is not NULL.  dphi [n] and
 * dtheta [map->nterms] are device outputs; either may be NULL.  A term that
 * is not finite makes the outputs it reaches NaN.  The workspace holds
 * nnz + (1 + 3^(d-1)) n doubles and the reduction partials
 * (vct_adjoint_workspace_size, with nnz = nl->nnz).  When both dphi and
 * dtheta are wanted, dtheta is computed on a second stream of the calling
 * host thread (created on its first such call on the device, default
 * priority, kept until the process ends), forked from `stream` and joined
 * back into it by events: the outputs are complete in `stream` order as for
 * one stream.                                                                  */
int vct_apply_ops_adjoint(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                          const double* state64, uint32_t out_mask, const vct_map* map /* host */,
                          const double* proj, const double* u, double* dphi, double* dtheta, void* ws,
                          size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- bathymetry adjoint, reading R2 */

/* Workspace of vct_apply_ops_adjoint_r2: 3^(d-1) + npairs + 2 doubles per
 * particle (npairs = 3 in 2-D, 6 in 3-D), the reduction partials and a short
 * int32 list. */
size_t vct_adjoint_r2_workspace_size(int dim, int64_t n, int nterms);

/* Sensitivity of loss = sum_i (lap_i - g_i)^2 to the bathymetry coefficients
 * when the particles' PHYSICAL positions are held fixed, so that their
 * projected heights z^_j = alpha (z_j + beta) move with the bottom (Sec. 2.1,
 * Eq. VCT; vct_apply_ops_adjoint is the other reading, projected positions
 * fixed).  Every row's SPH(2) derivatives then change through the offsets
 * r^_ij, the correction matrix L_i and the moment matrix M_i (Sec. 3.1,
 * Eq. sec_SPH2), and c_trans through z + beta = z^ / alpha:
 *   dtheta_t = sum_i u_i (d c_trans_i / d coef_t)|_{z^} . D^_i
 *            + sum_k (d loss / d z^_k) (d z^_k / d coef_t)|_{z},
 *   d loss / d z^_k = sum_{i in S_k + k} u_i d lap_i / d z^_k,
 * with the row derivatives by implicit differentiation of the SPH(2) system
 * (each term a function of one offset, summed in the push form of
 * vct_apply_ops_adjoint: exact integer sums, the same bits on every run).
 * Field values, volumes and the target stay fixed; d loss / d phi does not
 * change between the readings (vct_apply_ops_adjoint gives it).
 *   state64   vct_moments state whose out_mask holds LAP, PGRAD and PHESS
 *             (and not VCT_OPT_GRAD1: the system's own second-order gradient)
 *   proj      [n][n_out] FP64 vct_apply_ops output of phi with that mask
 *   phi [n], u [n] = 2 (lap - g)
 *   dtheta    [map->nterms] or NULL;  dzhat [n] or NULL: d loss / d z^_k
 * Needs nl->col16 and the stored chunk windows nl->chunk_win (vct_neighbors);
 * nl->col and nl->col_t are not read.
 * Non-finite terms make the outputs they reach NaN.  Asynchronous.            */
int vct_apply_ops_adjoint_r2(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                             const double* state64, uint32_t out_mask, const vct_map* map /* host */,
                             const double* proj, const double* phi, const double* u, double* dtheta, double* dzhat,
                             void* ws, size_t ws_bytes, void* stream);

/* Projected positions of physical points (Sec. 2.1, Eq. VCT): x^ = x,
 * y^ = y, z^ = alpha (z + beta); phys and proj SoA [dim][n] (distinct
 * buffers), any order.  Asynchronous.                                         */
int vct_map_project(int dim, int64_t n, const double* phys, const vct_map* map /* host */, double* proj,
                    void* stream);

/* ---------------------------------------------------------------- pressure step (Sec. 3.3) */

/* The pressure step of the projection method through the VCT (paper
 * Sec. 3.3, Eqs. VCT_ppe, VCT_ppe_w and the corrector of VCT_predictor).
 * `state64` comes from vct_moments with `out_mask` containing VCT_OUT_LAP
 * (VCT_OUT_LAP alone is enough; the first-order correction matrix at the
 * head of every state is what the divergence and gradient use).  Vector
 * fields are [dim][n] along the physical axes (2-D: x, z), in sorted order.
 *
 * vct_ppe_rhs: right-hand side of the pressure Poisson equation
 *   rhs_i = rho / dt * div_i + gamma * (rho * jr_i - dens_i) / dt^2
 * with
 *   div_i  = sum_{I,K} J_IK <d v*_I / d x^_K>^(1)_i: the physical divergence
 *            through the first-order projected gradients (Eqs. div_1st,
 *            jacobi; the printed "J <div^ v*>" is read this way);
 *   dens_i = rho * (V_i w(0) + sum_{j in S_i} V_j w_ij): the numerical density
 *            in the projected space (normalised kernel of unit integral);
 *   jr_i   = Jbar_i / J_i of Eq. VCT_ppe_w (NULL: 1, Eq. VCT_ppe).
 * Rows with dirichlet[i] != 0 get rhs_i = pbc[i] (pbc NULL: 0).  div and dens
 * (may be NULL) receive the two terms.  Particles with a NaN state get NaN.
 * Asynchronous.                                                               */
int vct_ppe_rhs(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                const double* state64, uint32_t out_mask, const vct_map* map /* host */, const double* vstar,
                double rho, double dt, double gamma, const double* jr, const uint8_t* dirichlet, const double* pbc,
                double* rhs, double* div, double* dens, void* stream);

/* vct_ppe_correct: v = v* - dt / rho * J <grad^ p>^(1) (Eqs. gra_1st and
 * grad_VCT: the first-order pressure gradient, as the paper's ISPH(2) uses),
 * vout [dim][n].  Asynchronous.                                               */
int vct_ppe_correct(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                    const double* state64, uint32_t out_mask, const vct_map* map /* host */, const double* p,
                    const double* vstar, double rho, double dt, double* vout, void* stream);

size_t vct_ppe_workspace_size(int dim, int64_t n, uint32_t out_mask);

/* vct_ppe_solve: the pressure Poisson equation c_trans . <D^ p>_i = rhs_i
 * (Eq. VCT_ppe) on rows with dirichlet[i] == 0 and p_i = rhs_i on the others
 * (dirichlet may be NULL), by BiCGSTAB with the Jacobi preconditioner on the
 * right (diagonal: the coefficient of p_i in row i).  The operator is
 * matrix-free: the FP64 Laplacian of vct_apply_ops on the fixed state.  `p`
 * holds the initial guess on entry and the solution on return.  Stops when
 * ||r|| <= tol ||rhs|| (the recurrence residual) or after max_iter
 * iterations.  The scalars of the method stay on the device; every inner
 * product is a fixed-order sum, so a solve gives the same bits on every run.
 * *iters (host, may be NULL) receives the iterations taken and *relres (host,
 * may be NULL) the true relative residual ||rhs - A p|| / ||rhs||.  Returns
 * VCT_OK when converged, VCT_W_NOCONV when it stopped on max_iter or a
 * breakdown.  SYNC (reads the scalars every 8 iterations).                    */
int vct_ppe_solve(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                  const double* state64, uint32_t out_mask, const uint8_t* dirichlet, const double* rhs, double* p,
                  double tol, int max_iter, int* iters /* host */, double* relres /* host */, void* ws,
                  size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- conventional ISPH operators */

/* The operators of the standard ISPH case of Table case_names, for comparison
 * with SPH(2) on the same particles.  Neither needs vct_moments (no correction
 * matrix).  Kernel gradient grad w_ij = -w'(r) r_ij / r, r_ij = r^_j - r^_i,
 * of the normalised kernel (unit integral); outputs [nf][n][n_out] in sorted
 * order, rows in the order of the mask as for vct_apply_ops.  A particle with
 * a neighbour at zero distance, a non-finite position, or where the mapping is
 * invalid (alpha not positive and finite) gets NaN outputs.  Asynchronous.
 *
 * vct_apply_ops0: the 0th-order models of Sec. 3.1 in the projected space,
 *   grad^ phi_i   = sum_j V_j phi_ij grad w_ij
 *   H^_IJ phi_i   = sum_j V_j (c r_ij^I r_ij^J / |r_ij|^2 - delta_IJ)
 *                             (r_ij . grad w_ij / |r_ij|^2) phi_ij
 *                   with c = 4 (2-D), 5 (3-D)             (Eq. sec_0th)
 * mapped like the SPH(2) derivatives: GRAD = J grad^, LAP = c_trans . D^,
 * CROSS and HESS = J H^ J^T + (d phi / d z^) (d2 z^)  (Eqs. grad_VCT, lap_VCT);
 * PGRAD, PHESS and PZ are the projected values.  Under the identity map LAP is
 * the trace of H^, which equals the Brookshaw Laplacian
 * 2 sum_j V_j (r_ij . grad w_ij / |r_ij|^2) phi_ij of Sec. 3.1 (the weights
 * c r^I r^I / |r|^2 - 1 sum to c - d = 2).  out_mask: any of GRAD, LAP, CROSS,
 * HESS, PGRAD, PHESS, PZ (VCT_OPT_GRAD1 is an SPH(2) option: VCT_E_ARG).     */
int vct_apply_ops0(const vct_nlist* nl, int nf, const double* phi_sorted, const double* pos_sorted,
                   const double* vol_sorted, int kernel, const vct_map* map /* host */, uint32_t out_mask,
                   double* out, void* stream);

/* vct_grad_sum: the summation pressure gradient (Eq. gra_sum) in the projected
 * space and its physical form (Eq. grad_VCT),
 *   grad^ p_i = rho_i sum_j m_j (p_j / rho_j^2 + p_i / rho_i^2) grad w_ij,
 *   m_j = rho_j V_j,
 * with rho [n] per particle, or rho_j = rho0 for all j when rho is NULL
 * (rho0 must then be finite and non-zero).  out_mask: GRAD (J grad^ p) and/or
 * PGRAD (grad^ p); out [n][n_out].                                            */
int vct_grad_sum(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted, int kernel,
                 const vct_map* map /* host */, const double* rho, double rho0, const double* p, uint32_t out_mask,
                 double* out, void* stream);

/* ---------------------------------------------------------------- volume smoothing (Sec. 3.6) */

/* The Jacobian determinant J = det J = alpha of the mapping (Sec. 2.1,
 * Eq. det_jacobi) at n points pos (SoA [dim][n], projected; any order):
 * J^N for vct_jbar_smooth and for the ratio Jbar / J of vct_ppe_rhs.  alpha
 * [n] device output.  Asynchronous.                                         */
int vct_map_alpha(int dim, int64_t n, const double* pos, const vct_map* map /* host */, double* alpha, void* stream);

/* Workspace of vct_jbar_smooth: n doubles. */
size_t vct_jbar_workspace_size(int64_t n);

/* The smoothed Jacobian determinant Jbar^N of the sigma method (paper
 * Sec. 3.6, Eq. VCT_bar_a), used by Eq. VCT_ppe_w (jr = Jbar / J of
 * vct_ppe_rhs).  With V_i = J_i / Jbar_i V, each neighbour pair (i, j)
 * exchanges the volume
 *   dJ_ij V,  dJ_ij = cv (re - |r^_ij|) / re (J_j / Jbar_j - J_i / Jbar_i),
 *   Jbar_i <- J_i Jbar_i / (J_i + Jbar_i dJ_ij),
 *   Jbar_j <- J_j Jbar_j / (J_j - Jbar_j dJ_ij),
 * along the neighbours j of each target particle i in turn, each update seen
 * by the next; every particle is a target once (so each pair is visited from
 * both ends).  The paper leaves the order of the targets open; here it is:
 * cells in 3^d phases, the cell with coordinates (cx, [cy,] cz) in phase
 * (cx mod 3) + 3 (cy mod 3) + 9 (cz mod 3) (2-D: (cx mod 3) + 3 (cz mod 3)),
 * phases in increasing order, the targets of a cell in sorted order, the
 * neighbours of a target in the order of its row.  Cells of one phase touch
 * disjoint particles, so they run in parallel; the result is that of the
 * sequential update in this order, up to rounding (the exchanges are formed
 * as J / Jbar values and a prefix scan over each row).
 *   J     [n]  Jacobian determinant J^N (alpha of the mapping, Eq. det_jacobi)
 *   jbar  [n]  in: Jbar^(N-1); out: Jbar^N (in place)
 *   cv         C_V (finite); re: r_e > 0 (normally the support radius nl->R)
 * Needs the neighbour lists (col16, chunk table) of vct_neighbors on the same
 * pos_sorted.  Non-finite J or Jbar propagate NaN to the particles they reach.
 * Asynchronous.                                                               */
int vct_jbar_smooth(const vct_nlist* nl, const double* pos_sorted, const double* J, double* jbar, double cv,
                    double re, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- allocation-free adjoint */

/* Size of the library's own scratch for vct_apply_ops_adjoint_noalloc. */
#define VCT_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * computation as vct_apply_ops_adjoint in its push form (nl->col_t is
 * ignored; nl->chunk_win is required when dphi is requested), with the
 * workspace taken from a fixed scratch array inside the library instead of a
 * caller buffer.  The caller still passes every input and output.  No device
 * memory is allocated or freed, and no allocating library routine is called.
 *   - Limit: vct_adjoint_workspace_size(dim, n, 0, nterms) must not exceed
 *     VCT_NOALLOC_SCRATCH_BYTES (64 MiB: about 830,000 particles in 3-D and
 *     2,000,000 in 2-D); larger sets return VCT_E_CAPACITY before any HIP
 *     call.
 *   - The scratch of the CURRENT device is used (the stream must belong to
 *     it).  Each device holds one copy for the life of the process; its
 *     address is looked up on the first call on that device.
 *   - Every call on one device shares that device's scratch, and a call
 *     leaves its contents behind (the next call clears what it needs).  Calls
 *     that overlap on one device race: serialise them (one stream, or events).
 * Results are bit-identical to vct_apply_ops_adjoint's push form on the same
 * inputs.                                                                      */
int vct_apply_ops_adjoint_noalloc(const vct_nlist* nl, const double* pos_sorted, const double* vol_sorted,
                                  int kernel, const double* state64, uint32_t out_mask, const vct_map* map /* host */,
                                  const double* proj, const double* u, double* dphi, double* dtheta, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* VCT_H */
