// Host-side helpers of the C ABI: status strings, error text, map validation,
// layout queries.
#include <string.h>

#include "common.h"
#include "map_dev.h"

namespace vct {

static thread_local char g_last_error[256] = "no error";

void set_last_error(hipError_t e) {
    const char* s = hipGetErrorString(e);
    strncpy(g_last_error, s ? s : "unknown HIP error", sizeof(g_last_error) - 1);
    g_last_error[sizeof(g_last_error) - 1] = '\0';
}

int map_params_from(const vct_map* m, int dim, MapParams& p) {
    memset(&p, 0, sizeof(p));
    if (!m) return VCT_E_ARG;
    if (m->kind < VCT_MAP_IDENTITY || m->kind > VCT_MAP_SIGMA) return VCT_E_ARG;
    if (m->nterms < 0 || m->nterms > VCT_MAX_TERMS || (m->nterms > 0 && !m->terms)) return VCT_E_ARG;
    p.kind = m->kind;
    p.nterms = m->nterms;
    p.dim = dim;
    p.Hhat = m->Hhat;
    p.H = m->H;
    p.dmin = m->dmin;
    p.eps = m->eps;
    if (m->kind == VCT_MAP_E || m->kind == VCT_MAP_BFE) {
        if (!(m->H > 0.0) || !(m->Hhat > 0.0) || !isfinite(m->H) || !isfinite(m->Hhat)) return VCT_E_ARG;
    }
    if (m->kind == VCT_MAP_SIGMA) {
        if (!(m->Hhat > 0.0) || !isfinite(m->Hhat) || !isfinite(m->H) || !(m->dmin >= 0.0) || !(m->eps >= 0.0))
            return VCT_E_ARG;
        p.limiter = (m->dmin > 0.0 || m->eps > 0.0) ? 1 : 0;
    }
    for (int t = 0; t < m->nterms; ++t) {
        const vct_term& tr = m->terms[t];
        if (tr.bx < VCT_BASIS_ONE || tr.bx > VCT_BASIS_SIN || tr.by < VCT_BASIS_ONE || tr.by > VCT_BASIS_SIN)
            return VCT_E_ARG;
        if (!isfinite(tr.coef) || !isfinite(tr.fx) || !isfinite(tr.fy)) return VCT_E_ARG;
        p.coef[t] = tr.coef;
        p.bx[t] = tr.bx;
        p.by[t] = tr.by;
        p.fx[t] = tr.fx;
        p.fy[t] = tr.fy;
    }
    return VCT_OK;
}

}  // namespace vct

using namespace vct;

extern "C" const char* vct_status_string(int status) {
    switch (status) {
    case VCT_OK: return "VCT_OK";
    case VCT_W_FLAGGED: return "VCT_W_FLAGGED: some particles were flagged (NaN outputs)";
    case VCT_E_ARG: return "VCT_E_ARG: invalid argument";
    case VCT_E_HIP: return "VCT_E_HIP: HIP runtime error";
    case VCT_E_CAPACITY: return "VCT_E_CAPACITY: output capacity too small";
    case VCT_E_NONFINITE: return "VCT_E_NONFINITE: non-finite input position";
    case VCT_E_WORKSPACE: return "VCT_E_WORKSPACE: workspace missing or too small";
    default: return "unknown status";
    }
}

extern "C" const char* vct_last_error(void) { return g_last_error; }

extern "C" int vct_n_out(int dim, uint32_t out_mask) {
    if ((dim != 2 && dim != 3) || !mask_valid(out_mask)) return 0;
    return n_out_rows(dim, out_mask);
}

extern "C" int vct_state_stride(int dim, uint32_t out_mask) {
    if ((dim != 2 && dim != 3) || !mask_valid(out_mask)) return 0;
    const int nL = dim == 2 ? 3 : 6, nk = dim == 2 ? 5 : 9;
    return nL + n_out_rows(dim, out_mask) * (nk + dim);
}
