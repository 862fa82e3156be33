/* Oracle for the VCT-SPH(2) derivative operators (test infrastructure only).
 * Private header of oracle/orc.c; the GPU library never includes it. */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

enum { ORC_B_ONE = 0, ORC_B_LIN = 1, ORC_B_COS = 2, ORC_B_SIN = 3 };
enum { ORC_MAP_IDENTITY = 0, ORC_MAP_E = 1, ORC_MAP_BF = 2, ORC_MAP_BFE = 3, ORC_MAP_SIGMA = 4,
       ORC_MAP_PER_PARTICLE = 5 };
enum { ORC_K_WENDLAND = 0, ORC_K_SPLINE = 1 };

/* per-particle flag bits */
enum {
    ORC_F_FEW = 1,          /* fewer than d + m neighbours */
    ORC_F_SINGULAR_A = 2,   /* first-order correction matrix singular */
    ORC_F_SINGULAR_M = 4,   /* SPH(2) matrix M singular */
    ORC_F_NONFINITE = 8,    /* non-finite position or volume */
    ORC_F_DUPLICATE = 16,   /* a neighbour at zero distance */
    ORC_F_MAP = 32          /* alpha not finite or not positive (Sec. 2.1 needs alpha > 0) */
};

#define ORC_PIVOT_TOL 1e-12

/* Output record per (particle, field):
 *  [0:3]  physical gradient (x, y, z)       [3] physical Laplacian (c_trans . D^)
 *  [4:7]  physical cross derivatives xy, xz, yz
 *  [7:13] physical Hessian xx, yy, zz, xy, xz, yz
 *  [13:16] first-order projected gradient    [16:19] second-order projected gradient
 *  [19:25] SPH(2) vector D (xx, yy, zz, 2xy, 2xz, 2yz) in the projected space
 *  [25:31] D^ = [dz^, xx, yy, zz, xz, yz] in the projected space
 *  [31]   physical Laplacian as the trace of the physical Hessian
 * 2-D (x, z) sets fill the x and z slots and leave every y slot zero.        */
#define ORC_REC 32

typedef struct {
    int kind;
    double Hhat, H, dmin, eps;
    int nterms;
    const double* terms;     /* nterms x 5: coef, bx, fx, by, fy */
} orc_map;

#endif
