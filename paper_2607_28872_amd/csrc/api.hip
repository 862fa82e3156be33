// Host-side helpers of the C ABI: status strings, error text, map validation,
// layout queries, launch timing.
#include <string.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "common.h"
#include "map_dev.h"

namespace vct {

static thread_local char g_last_error[256] = "no error";

void set_last_error(hipError_t e) {
    const char* s = hipGetErrorString(e);
    strncpy(g_last_error, s ? s : "unknown HIP error", sizeof(g_last_error) - 1);
    g_last_error[sizeof(g_last_error) - 1] = '\0';
}

// Index of the factor (kind, frequency) of one axis in the separable table,
// inserted when new; -1 if the table is full.
static int sep_factor(int kind, double f, int32_t* fkind, int32_t* fslot, double* freq, int32_t& nf,
                      int32_t& nq) {
    int q = 0;
    if (kind == VCT_BASIS_COS || kind == VCT_BASIS_SIN) {
        q = -1;
        for (int j = 0; j < nq; ++j)
            if (freq[j] == f) q = j;
        if (q < 0) {
            if (nq == kMapFq) return -1;
            q = nq;
            freq[nq++] = f;
        }
    }
    for (int a = 0; a < nf; ++a)
        if (fkind[a] == kind && fslot[a] == q) return a;
    if (nf == kMapFn) return -1;
    fkind[nf] = kind;
    fslot[nf] = q;
    return nf++;
}

// The separable table of the bottom terms (sep = 0 when it does not fit).
static void build_separable(MapParams& p) {
    p.sep = 0;
    p.nfx = p.nfy = p.nqx = p.nqy = 0;
    for (int t = 0; t < p.nterms; ++t) {
        const int a = sep_factor(p.bx[t], p.fx[t], p.fx_kind, p.fx_q, p.qx, p.nfx, p.nqx);
        const int b = sep_factor(p.by[t], p.fy[t], p.fy_kind, p.fy_q, p.qy, p.nfy, p.nqy);
        if (a < 0 || b < 0) {
            memset(p.cm, 0, sizeof(p.cm));
            p.nfx = p.nfy = p.nqx = p.nqy = 0;
            return;
        }
        p.cm[a][b] += p.coef[t];
        p.term_a[t] = a;
        p.term_b[t] = b;
    }
    p.sep = 1;
}

int map_params_from(const vct_map* m, int dim, int64_t n, MapParams& p) {
    memset(&p, 0, sizeof(p));
    if (!m) return VCT_E_ARG;
    if (m->kind < VCT_MAP_IDENTITY || m->kind > VCT_MAP_PER_PARTICLE) return VCT_E_ARG;
    if (m->nterms < 0 || m->nterms > VCT_MAX_TERMS || (m->nterms > 0 && !m->terms)) return VCT_E_ARG;
    if (m->kind == VCT_MAP_PER_PARTICLE) {
        // the table replaces the bottom terms; it must cover every point of the call
        if (m->nterms != 0 || m->coef_n != n || (n > 0 && !m->coef)) return VCT_E_ARG;
        p.pp = m->coef;
        p.pp_n = m->coef_n;
    }
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
        // a limiter with eps = 0 is a hard max(D, dmin): its second derivative
        // is 0/0 where D = dmin, so the smooth limiter needs eps > 0
        if (m->dmin > 0.0 && !(m->eps > 0.0)) return VCT_E_ARG;
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
    build_separable(p);
    return VCT_OK;
}

// ------------------------------------------------------------------ launch timing

namespace {
struct TimingRec {
    const char* name;
    hipEvent_t a, b;
    bool closed;
};
struct TimingAgg {
    const char* name;
    int64_t launches;
    double ms;
};
std::atomic<bool> g_timing{false};
std::mutex g_tmu;
std::vector<TimingRec> g_pending;
std::vector<hipEvent_t> g_free_events;
std::vector<TimingAgg> g_agg;

hipEvent_t take_event() {
    if (!g_free_events.empty()) {
        hipEvent_t e = g_free_events.back();
        g_free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

void drop_pending() {
    for (TimingRec& r : g_pending) {
        if (r.a) g_free_events.push_back(r.a);
        if (r.b) g_free_events.push_back(r.b);
    }
    g_pending.clear();
}

// Waits for every closed record and adds its duration to its kernel's total.
void fold_pending() {
    for (TimingRec& r : g_pending) {
        if (!r.closed || !r.a || !r.b) continue;
        float ms = 0.0f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
        size_t k = 0;
        while (k < g_agg.size() && strcmp(g_agg[k].name, r.name) != 0) ++k;
        if (k == g_agg.size()) g_agg.push_back({r.name, 0, 0.0});
        g_agg[k].launches += 1;
        g_agg[k].ms += ms;
    }
    drop_pending();
}
}  // namespace

bool timing_on() { return g_timing.load(std::memory_order_relaxed); }

int timing_begin(const char* name, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_tmu);
    hipEvent_t a = take_event(), b = take_event();
    if (!a || !b || hipEventRecord(a, s) != hipSuccess) {
        if (a) g_free_events.push_back(a);
        if (b) g_free_events.push_back(b);
        return -1;
    }
    g_pending.push_back({name, a, b, false});
    return (int)g_pending.size() - 1;
}

void timing_end(int rec, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (rec < 0 || rec >= (int)g_pending.size()) return;
    g_pending[rec].closed = hipEventRecord(g_pending[rec].b, s) == hipSuccess;
}

VCT_CHECKS_TU(checks_api)

}  // namespace vct

using namespace vct;

extern "C" int vct_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_tmu);
    const bool was = g_timing.exchange(on != 0);
    if (was && !on) fold_pending();
    return was ? 1 : 0;
}

extern "C" void vct_timing_reset(void) {
    std::lock_guard<std::mutex> lk(g_tmu);
    drop_pending();
    g_agg.clear();
}

extern "C" int vct_timing_count(void) {
    std::lock_guard<std::mutex> lk(g_tmu);
    fold_pending();
    return (int)g_agg.size();
}

extern "C" int vct_timing_get(int idx, const char** name, int64_t* launches, double* total_ms) {
    std::lock_guard<std::mutex> lk(g_tmu);
    fold_pending();
    if (idx < 0 || idx >= (int)g_agg.size() || !name || !launches || !total_ms) return VCT_E_ARG;
    *name = g_agg[idx].name;
    *launches = g_agg[idx].launches;
    *total_ms = g_agg[idx].ms;
    return VCT_OK;
}

namespace vct {
int checks_adjoint(uint32_t*);
int checks_apply(uint32_t*);
int checks_cells(uint32_t*);
int checks_isph(uint32_t*);
int checks_jbar(uint32_t*);
int checks_moments(uint32_t*);
int checks_ppe(uint32_t*);
}  // namespace vct

extern "C" int vct_device_checks(uint32_t* bits) {
    if (!bits) return VCT_E_ARG;
    *bits = 0;
    VCT_HIP_CHECK(hipDeviceSynchronize());
    int (*const take[])(uint32_t*) = {checks_api, checks_adjoint, checks_apply, checks_cells,
                                      checks_isph, checks_jbar, checks_moments, checks_ppe};
    for (auto f : take) {
        const int st = f(bits);
        if (st) return st;
    }
    return VCT_DEVICE_CHECKS ? 1 : 0;
}

extern "C" const char* vct_status_string(int status) {
    switch (status) {
    case VCT_OK: return "VCT_OK";
    case VCT_W_FLAGGED: return "VCT_W_FLAGGED: some particles were flagged (NaN outputs)";
    case VCT_W_NOCONV: return "VCT_W_NOCONV: the iterative solve stopped before its tolerance";
    case VCT_E_ARG: return "VCT_E_ARG: invalid argument";
    case VCT_E_HIP: return "VCT_E_HIP: HIP runtime error";
    case VCT_E_CAPACITY: return "VCT_E_CAPACITY: output capacity too small";
    case VCT_E_NONFINITE: return "VCT_E_NONFINITE: non-finite input position";
    case VCT_E_WORKSPACE: return "VCT_E_WORKSPACE: workspace missing or too small";
    case VCT_E_WINDOW: return "VCT_E_WINDOW: a neighbour window exceeds 65535 particles";
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
