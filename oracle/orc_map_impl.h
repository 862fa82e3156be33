/* Oracle: vertical coordinate transformation coefficients, templated over the
 * scalar type so that the same statements serve the real evaluation and the
 * complex-step derivative with respect to a bathymetry coefficient.
 *
 * Test infrastructure only (see orc.c).  Included twice from orc.c with
 *   ORC_T      scalar type (double / double complex)
 *   ORC_SQRT   square root for ORC_T
 *   ORC_FN(x)  name mangling
 *
 * Mapping (paper Sec. 2.1, Eq. VCT): x^ = x, y^ = y, z^ = alpha(x,y) (z + beta(x,y)).
 * Choices of alpha and beta (paper Sec. 2.2):
 *   identity : alpha = 1,                beta = 0
 *   E-SPH    : alpha = Hhat / H,         beta = 0
 *   BF-SPH   : alpha = 1,                beta = -h
 *   BFE-SPH  : alpha = Hhat / H,         beta = -h
 *   sigma-SPH: alpha = Hhat / (H - h),   beta = -h
 *   per-particle: alpha, beta and their derivatives given at every point
 *              (any transformation of the form of Eq. VCT)
 * For sigma-SPH the depth D = H - h is limited from below (the paper asks for
 * a constant alpha outside the applicable range without giving the range); the
 * reading used here replaces D by the smooth maximum
 *   D_eff = ( D + dmin + sqrt((D - dmin)^2 + eps^2) ) / 2
 * in both alpha = Hhat / D_eff and beta = D_eff - H (so beta = -h where the
 * limiter is inactive).
 */

/* h and its first and second horizontal derivatives at (x, y).  The term
 * coefficient `t_pert` (if >= 0) gets the extra (complex) increment `dc`. */
static void ORC_FN(bottom)(const double* terms, int nterms, int dim, double x, double y,
                           int t_pert, ORC_T dc, ORC_T hv[6])
{
    for (int k = 0; k < 6; ++k) hv[k] = 0;
    for (int t = 0; t < nterms; ++t) {
        const double* tr = terms + 5 * t;
        ORC_T c = tr[0];
        if (t == t_pert) c = c + dc;
        double bx[3], by[3];
        orc_basis((int)tr[1], tr[2], x, bx);
        orc_basis((int)tr[3], tr[4], y, by);
        if (dim == 2) { by[1] = 0; by[2] = 0; }   /* 2-D: h depends on x only */
        hv[0] += c * bx[0] * by[0];   /* h    */
        hv[1] += c * bx[1] * by[0];   /* h_x  */
        hv[2] += c * bx[0] * by[1];   /* h_y  */
        hv[3] += c * bx[2] * by[0];   /* h_xx */
        hv[4] += c * bx[1] * by[1];   /* h_xy */
        hv[5] += c * bx[0] * by[2];   /* h_yy */
    }
}

/* alpha, beta and their derivatives:
 *   ab[0..5]  = alpha, alpha_x, alpha_y, alpha_xx, alpha_xy, alpha_yy
 *   ab[6..11] = beta,  beta_x,  beta_y,  beta_xx,  beta_xy,  beta_yy      */
static void ORC_FN(alpha_beta)(const orc_map* mp, int dim, double x, double y, int64_t idx, int t_pert,
                               ORC_T dc, ORC_T ab[12])
{
    for (int k = 0; k < 12; ++k) ab[k] = 0;
    ab[0] = 1;
    if (mp->kind == ORC_MAP_IDENTITY) return;
    if (mp->kind == ORC_MAP_PER_PARTICLE) {
        /* given at every point (point idx of the table orc_set_per_particle set) */
        for (int k = 0; k < 12; ++k)
            ab[k] = (g_orc_pp && idx >= 0 && idx < g_orc_pp_n) ? g_orc_pp[k * g_orc_pp_n + idx] : NAN;
        if (dim == 2) { ab[2] = 0; ab[4] = 0; ab[5] = 0; ab[8] = 0; ab[10] = 0; ab[11] = 0; }
        return;
    }
    if (mp->kind == ORC_MAP_E) { ab[0] = mp->Hhat / mp->H; return; }
    ORC_T h[6];
    ORC_FN(bottom)(mp->terms, mp->nterms, dim, x, y, t_pert, dc, h);
    if (mp->kind == ORC_MAP_BF || mp->kind == ORC_MAP_BFE) {
        ab[0] = (mp->kind == ORC_MAP_BF) ? 1.0 : mp->Hhat / mp->H;
        for (int k = 0; k < 6; ++k) ab[6 + k] = -h[k];
        return;
    }
    /* sigma-SPH with the smooth depth limiter */
    ORC_T D = mp->H - h[0];
    ORC_T Dx = -h[1], Dy = -h[2], Dxx = -h[3], Dxy = -h[4], Dyy = -h[5];
    ORC_T E, s1, s2;
    if (mp->eps > 0 || mp->dmin > 0) {
        ORC_T S = ORC_SQRT((D - mp->dmin) * (D - mp->dmin) + mp->eps * mp->eps);
        E = 0.5 * (D + mp->dmin + S);
        s1 = 0.5 * (1.0 + (D - mp->dmin) / S);
        s2 = 0.5 * mp->eps * mp->eps / (S * S * S);
    } else {
        E = D; s1 = 1; s2 = 0;
    }
    ORC_T Ex = s1 * Dx, Ey = s1 * Dy;
    ORC_T Exx = s2 * Dx * Dx + s1 * Dxx;
    ORC_T Exy = s2 * Dx * Dy + s1 * Dxy;
    ORC_T Eyy = s2 * Dy * Dy + s1 * Dyy;
    ORC_T Hh = mp->Hhat;
    ab[0] = Hh / E;
    ab[1] = -Hh * Ex / (E * E);
    ab[2] = -Hh * Ey / (E * E);
    ab[3] = Hh * (2.0 * Ex * Ex / (E * E * E) - Exx / (E * E));
    ab[4] = Hh * (2.0 * Ex * Ey / (E * E * E) - Exy / (E * E));
    ab[5] = Hh * (2.0 * Ey * Ey / (E * E * E) - Eyy / (E * E));
    ab[6] = E - mp->H;
    ab[7] = Ex; ab[8] = Ey; ab[9] = Exx; ab[10] = Exy; ab[11] = Eyy;
}

/* Coefficients of the physical-space derivatives at a particle with projected
 * position (x, y, zh):
 *   Jm[3][3]  Jacobian in the paper's layout (Eq. jacobi): Jm[I][K] = d r^_K / d r_I
 *   ct[6]     Laplacian coefficient vector c_trans (Eq. lap_VCT), acting on
 *             D^ = [d/dz^, d2/dx^2, d2/dy^2, d2/dz^2, d2/dx^dz^, d2/dy^dz^]
 *   hz[3][3]  second derivatives of z^ with respect to physical (x, y, z)
 * z + beta is recovered from the projected height as zh / alpha.  In 2-D the
 * vertical plane (x, z) is used: y = 0 and every y-derivative vanishes.    */
static void ORC_FN(map_coeffs)(const orc_map* mp, int dim, double x, double y, double zh, int64_t idx,
                               int t_pert, ORC_T dc,
                               ORC_T Jm[3][3], ORC_T ct[6], ORC_T hz[3][3])
{
    ORC_T ab[12];
    ORC_FN(alpha_beta)(mp, dim, x, y, idx, t_pert, dc, ab);
    ORC_T a = ab[0], ax = ab[1], ay = ab[2], axx = ab[3], axy = ab[4], ayy = ab[5];
    ORC_T bx = ab[7], by = ab[8], bxx = ab[9], bxy = ab[10], byy = ab[11];
    ORC_T zb = zh / a;                        /* z + beta */
    ORC_T gx = ax * zb + a * bx;              /* d z^ / dx */
    ORC_T gy = ay * zb + a * by;              /* d z^ / dy */
    for (int I = 0; I < 3; ++I) for (int K = 0; K < 3; ++K) Jm[I][K] = 0;
    Jm[0][0] = 1; Jm[1][1] = 1;
    Jm[0][2] = gx; Jm[1][2] = gy; Jm[2][2] = a;
    ct[0] = (axx + ayy) * zb + 2.0 * (ax * bx + ay * by) + a * (bxx + byy);
    ct[1] = 1;
    ct[2] = 1;
    ct[3] = a * a + gx * gx + gy * gy;
    ct[4] = 2.0 * gx;
    ct[5] = 2.0 * gy;
    hz[0][0] = axx * zb + 2.0 * ax * bx + a * bxx;
    hz[1][1] = ayy * zb + 2.0 * ay * by + a * byy;
    hz[0][1] = hz[1][0] = axy * zb + ax * by + ay * bx + a * bxy;
    hz[0][2] = hz[2][0] = ax;
    hz[1][2] = hz[2][1] = ay;
    hz[2][2] = 0;
}

/* c_trans (Eq. lap_VCT) at a point whose projected height zh is itself of the
 * scalar type, for complex-step derivatives in which both the bathymetry
 * coefficient t_pert and z^ carry an imaginary part (physical positions held
 * fixed, so z^ moves with the bottom).  Same statements as map_coeffs. */
static void ORC_FN(map_ct)(const orc_map* mp, int dim, double x, double y, ORC_T zh, int64_t idx, int t_pert,
                           ORC_T dc, ORC_T ct[6])
{
    ORC_T ab[12];
    ORC_FN(alpha_beta)(mp, dim, x, y, idx, t_pert, dc, ab);
    ORC_T a = ab[0], ax = ab[1], ay = ab[2], axx = ab[3], ayy = ab[5];
    ORC_T bx = ab[7], by = ab[8], bxx = ab[9], byy = ab[11];
    ORC_T zb = zh / a;                        /* z + beta */
    ORC_T gx = ax * zb + a * bx;
    ORC_T gy = ay * zb + a * by;
    ct[0] = (axx + ayy) * zb + 2.0 * (ax * bx + ay * by) + a * (bxx + byy);
    ct[1] = 1;
    ct[2] = 1;
    ct[3] = a * a + gx * gx + gy * gy;
    ct[4] = 2.0 * gx;
    ct[5] = 2.0 * gy;
}
