// C ABI of libgammax: argument checks, the per-context workspace and cell-table cache,
// and the device pipeline of one gamma map (Algorithm A2 steps 2-7).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "gammax.h"
#include "internal.hpp"

using namespace gammax;

struct gammax_ctx {
    int device = 0;
    std::string err;
    // per-call scalars
    Scalars* d_sc = nullptr;
    Scalars* h_sc = nullptr;  // pinned
    unsigned long long* d_cnt = nullptr;
    unsigned long long* h_cnt = nullptr;  // pinned
    uint32_t* d_count = nullptr;
    uint32_t* h_count = nullptr;  // pinned
    // node work list and sort scratch
    uint32_t *keys = nullptr, *vals = nullptr, *tkeys = nullptr, *tvals = nullptr;
    int64_t item_cap = 0;
    uint32_t* blockcnt = nullptr;
    int64_t blk_cap = 0;
    uint32_t* hist = nullptr;
    int64_t hist_cap = 0;
    // cell table cache
    TabEntry* tab = nullptr;
    int64_t tab_cap = 0;
    int64_t tab_len = 0;
    bool tab_valid = false;
    TableGeom tab_geom{};
    uint32_t *tb_keys = nullptr, *tb_vals = nullptr, *tb_tk = nullptr, *tb_tv = nullptr;
    int64_t tb_cap = 0;
    uint32_t* tb_hist = nullptr;
    int64_t tb_hist_cap = 0;
    hipEvent_t ev[8] = {};
    bool events = false;
};

namespace {

// Largest candidate box the table builder accepts (entries of the unsorted box).
constexpr int64_t kMaxTableBox = (int64_t)1 << 28;

const char* kStatusText[] = {
    "ok",
    "null pointer",
    "bad shape (ndim must be 2 or 3, every axis >= 2 nodes, < 2^31 nodes in total)",
    "bad parameter (spacing, DD, DTA must be finite and > 0; threshold in [0,1); options valid)",
    "non-finite dose value",
    "out of memory",
    "HIP runtime error",
    "search radius needs a larger cell table than the library allows",
    "global normalisation needs a positive reference dose",
};

gammax_status_t fail(gammax_ctx* c, gammax_status_t st, const std::string& why) {
    if (c) c->err = why;
    return st;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), (e_ == hipErrorOutOfMemory) ? GAMMAX_E_NOMEM : GAMMAX_E_DEVICE, \
                        std::string(#call) + ": " + hipGetErrorString(e_));                 \
    } while (0)

template <typename P>
gammax_status_t grow(gammax_ctx* c, P** p, int64_t* cap, int64_t need) {
    if (need <= *cap && *p) return GAMMAX_OK;
    if (*p) {
        hipError_t e = hipFree(*p);
        *p = nullptr;
        *cap = 0;
        if (e != hipSuccess) return fail(c, GAMMAX_E_DEVICE, std::string("hipFree: ") + hipGetErrorString(e));
    }
    int64_t n = need > 0 ? need : 1;
    hipError_t e = hipMalloc((void**)p, (size_t)n * sizeof(P));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, GAMMAX_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    *cap = n;
    return GAMMAX_OK;
}

// Four uint32 buffers of one capacity (keys, values and their sort ping-pong copies).
gammax_status_t grow4(gammax_ctx* c, uint32_t** a, uint32_t** b, uint32_t** d, uint32_t** e, int64_t* cap,
                      int64_t need) {
    if (need <= *cap && *a) return GAMMAX_OK;
    uint32_t** bufs[4] = {a, b, d, e};
    for (uint32_t** p : bufs) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    *cap = 0;
    const int64_t n = need > 0 ? need : 1;
    for (uint32_t** p : bufs) {
        hipError_t err = hipMalloc((void**)p, (size_t)n * sizeof(uint32_t));
        if (err != hipSuccess) {
            *p = nullptr;
            return fail(c, GAMMAX_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(err));
        }
    }
    *cap = n;
    return GAMMAX_OK;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

gammax_status_t check_problem(gammax_ctx* c, const gammax_problem_t* p, int64_t* n_out) {
    if (!p) return fail(c, GAMMAX_E_NULL, "problem is NULL");
    if (p->ndim != 2 && p->ndim != 3) return fail(c, GAMMAX_E_SHAPE, "ndim must be 2 or 3");
    int64_t n = 1;
    for (int i = 0; i < p->ndim; ++i) {
        if (p->shape[i] < 2) return fail(c, GAMMAX_E_SHAPE, "every axis needs at least 2 nodes");
        if (p->shape[i] > ((int64_t)1 << 30)) return fail(c, GAMMAX_E_SHAPE, "axis too long");
        n *= p->shape[i];
        if (n >= ((int64_t)1 << 31)) return fail(c, GAMMAX_E_SHAPE, "grid must hold < 2^31 nodes");
        if (!finite_pos(p->spacing_mm[i])) return fail(c, GAMMAX_E_PARAM, "spacing must be finite and > 0");
    }
    if (!finite_pos(p->dd)) return fail(c, GAMMAX_E_PARAM, "DD must be finite and > 0");
    if (!finite_pos(p->dta_mm)) return fail(c, GAMMAX_E_PARAM, "DTA must be finite and > 0");
    if (!(p->dose_threshold >= 0.0 && p->dose_threshold < 1.0))
        return fail(c, GAMMAX_E_PARAM, "dose_threshold must lie in [0, 1)");
    if (p->norm != GAMMAX_GLOBAL && p->norm != GAMMAX_LOCAL) return fail(c, GAMMAX_E_PARAM, "norm must be 0 or 1");
    *n_out = n;
    return GAMMAX_OK;
}

gammax_status_t check_options(gammax_ctx* c, const gammax_options_t* o) {
    if (o->sort_mode != GAMMAX_SORT_NONE && o->sort_mode != GAMMAX_SORT_DD)
        return fail(c, GAMMAX_E_PARAM, "unknown sort_mode");
    if (o->precision < GAMMAX_PREC_FP32 || o->precision > GAMMAX_PREC_FP64)
        return fail(c, GAMMAX_E_PARAM, "unknown precision");
    if (!(o->cond_threshold >= 1.0)) return fail(c, GAMMAX_E_PARAM, "cond_threshold must be >= 1");
    if (o->timing != 0 && o->timing != 1) return fail(c, GAMMAX_E_PARAM, "timing must be 0 or 1");
    for (int i = 0; i < 7; ++i)
        if (o->reserved[i] != 0) return fail(c, GAMMAX_E_PARAM, "reserved option fields must be 0");
    return GAMMAX_OK;
}

__global__ void k_zero_u32(uint32_t* p) {
    if (threadIdx.x == 0) *p = 0u;
}

bool same_geom(const TableGeom& a, const TableGeom& b) {
    if (a.ndim != b.ndim) return false;
    for (int i = 0; i < a.ndim; ++i)
        if (a.shape[i] != b.shape[i] || a.s[i] != b.s[i]) return false;
    return true;
}

// Build the sorted cell table for `g` into the context cache (synchronises `s`).
gammax_status_t build_table(gammax_ctx* c, TableGeom g, hipStream_t s) {
    table_box(g);
    if (g.box > kMaxTableBox)
        return fail(c, GAMMAX_E_RADIUS, "cell table candidate box of " + std::to_string(g.box) + " entries");
    c->tab_valid = false;
    gammax_status_t st;
    if ((st = grow4(c, &c->tb_keys, &c->tb_vals, &c->tb_tk, &c->tb_tv, &c->tb_cap, g.box)) != GAMMAX_OK) return st;
    if ((st = grow(c, &c->tb_hist, &c->tb_hist_cap, sort_hist_words(g.box))) != GAMMAX_OK) return st;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, c->d_count);
    HIPCHK(c, launch_table_gen(g, c->tb_keys, c->tb_vals, c->d_count, s));
    HIPCHK(c, radix_sort_pairs(c->tb_keys, c->tb_vals, c->tb_tk, c->tb_tv, g.box, c->tb_hist, s));
    HIPCHK(c, hipMemcpyAsync(c->h_count, c->d_count, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const int64_t T = *c->h_count;
    if ((st = grow(c, &c->tab, &c->tab_cap, T)) != GAMMAX_OK) return st;
    HIPCHK(c, launch_table_rows(g, c->tb_vals, T, c->tab, s));
    c->tab_len = T;
    c->tab_geom = g;
    c->tab_valid = true;
    return GAMMAX_OK;
}

TableGeom geom_of(const gammax_problem_t* p) {
    TableGeom g{};
    g.ndim = p->ndim;
    for (int i = 0; i < 3; ++i) {
        g.shape[i] = i < p->ndim ? p->shape[i] : 1;
        g.s[i] = i < p->ndim ? p->spacing_mm[i] / p->dta_mm : 1.0;
    }
    return g;
}

gammax_status_t ensure_events(gammax_ctx* c) {
    if (c->events) return GAMMAX_OK;
    for (auto& e : c->ev) HIPCHK(c, hipEventCreate(&e));
    c->events = true;
    return GAMMAX_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.0f;
    return ms;
}

}  // namespace

extern "C" {

void gammax_options_default(gammax_options_t* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->sort_mode = GAMMAX_SORT_DD;
    opt->precision = GAMMAX_PREC_GUARDED;
    opt->cond_threshold = 1e6;
    opt->timing = 0;
}

const char* gammax_status_string(gammax_status_t st) {
    int k = -(int)st;
    if (k < 0 || k >= (int)(sizeof(kStatusText) / sizeof(kStatusText[0]))) return "unknown status";
    return kStatusText[k];
}

const char* gammax_last_error(const gammax_ctx_t* ctx) { return ctx ? ctx->err.c_str() : ""; }

gammax_status_t gammax_ctx_create(int device, gammax_ctx_t** out) {
    if (!out) return GAMMAX_E_NULL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GAMMAX_E_DEVICE;
    gammax_ctx* c = new (std::nothrow) gammax_ctx();
    if (!c) return GAMMAX_E_NOMEM;
    c->device = device;
    if (hipSetDevice(device) != hipSuccess ||
        hipMalloc((void**)&c->d_sc, sizeof(Scalars)) != hipSuccess ||
        hipHostMalloc((void**)&c->h_sc, sizeof(Scalars), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&c->d_cnt, 3 * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc((void**)&c->h_cnt, 3 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&c->d_count, sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc((void**)&c->h_count, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        gammax_ctx_destroy(c);
        return GAMMAX_E_NOMEM;
    }
    *out = c;
    return GAMMAX_OK;
}

gammax_status_t gammax_ctx_destroy(gammax_ctx_t* c) {
    if (!c) return GAMMAX_OK;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    void* dev[] = {c->d_sc, c->d_cnt, c->d_count, c->keys, c->vals, c->tkeys, c->tvals, c->blockcnt,
                   c->hist, c->tab, c->tb_keys, c->tb_vals, c->tb_tk, c->tb_tv, c->tb_hist};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    void* host[] = {c->h_sc, c->h_cnt, c->h_count};
    for (void* p : host)
        if (p) (void)hipHostFree(p);
    if (c->events)
        for (auto& e : c->ev) (void)hipEventDestroy(e);
    delete c;
    return GAMMAX_OK;
}

gammax_status_t gammax_map(gammax_ctx_t* c, const gammax_problem_t* p, const gammax_options_t* opt_in,
                           const float* ref, const float* ev, float* gamma, gammax_result_t* res,
                           void* stream) {
    if (!c) return GAMMAX_E_NULL;
    if (!ref || !ev || !gamma || !res) return fail(c, GAMMAX_E_NULL, "dose, gamma and result pointers are required");
    int64_t n = 0;
    gammax_status_t st = check_problem(c, p, &n);
    if (st != GAMMAX_OK) return st;
    if ((const float*)gamma == ref || (const float*)gamma == ev)
        return fail(c, GAMMAX_E_PARAM, "gamma must not alias the dose arrays");
    gammax_options_t opt;
    if (opt_in) opt = *opt_in;
    else gammax_options_default(&opt);
    if ((st = check_options(c, &opt)) != GAMMAX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    std::memset(res, 0, sizeof(*res));

    // workspace
    if ((st = grow4(c, &c->keys, &c->vals, &c->tkeys, &c->tvals, &c->item_cap, n)) != GAMMAX_OK) return st;
    if ((st = grow(c, &c->blockcnt, &c->blk_cap, (n + PREP_TILE - 1) / PREP_TILE)) != GAMMAX_OK) return st;
    if ((st = grow(c, &c->hist, &c->hist_cap, sort_hist_words(n))) != GAMMAX_OK) return st;
    if (opt.timing && (st = ensure_events(c)) != GAMMAX_OK) return st;

    const bool local = p->norm == GAMMAX_LOCAL;
    // step 2 (Kernel 1): dose maximum, mask, gamma0, ordered compaction
    if (opt.timing) HIPCHK(c, hipEventRecord(c->ev[0], s));
    HIPCHK(c, launch_init_scalars(c->d_sc, s));
    HIPCHK(c, launch_dose_max(ref, ev, n, c->d_sc, s));
    PrepArgs pa{};
    pa.ref = ref;
    pa.ev = ev;
    pa.gamma = gamma;
    pa.n = n;
    pa.thr = (float)p->dose_threshold;
    pa.dd = (float)p->dd;
    pa.local = local ? 1 : 0;
    pa.sc = c->d_sc;
    pa.blockcnt = c->blockcnt;
    pa.keys = c->keys;
    pa.vals = c->vals;
    HIPCHK(c, launch_prep(pa, s));
    if (opt.timing) HIPCHK(c, hipEventRecord(c->ev[1], s));
    HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if (c->h_sc->flags & FLAG_NONFINITE) return fail(c, GAMMAX_E_NONFINITE, "a dose value is NaN or infinite");
    const float dmax = ord_to_float(c->h_sc->dmax_ord);
    if (!local && !(dmax > 0.0f)) return fail(c, GAMMAX_E_DOSE, "max reference dose is not positive");
    const uint32_t M = c->h_sc->n_masked;
    const float r2 = u2f(c->h_sc->r2_bits);

    // steps 4-5 (Kernel 2 + sort): the cell table, cached while it still covers the radius
    float ms_table = 0.0f;
    TableGeom g = geom_of(p);
    const bool need_walk = M > 0 && r2 > 0.0f;
    if (need_walk && !(c->tab_valid && same_geom(c->tab_geom, g) && c->tab_geom.r2_cap >= (double)r2)) {
        g.r2_cap = (double)r2 * 1.5;   // headroom so that nearby radii reuse the table
        if (opt.timing) HIPCHK(c, hipEventRecord(c->ev[2], s));
        if ((st = build_table(c, g, s)) != GAMMAX_OK) return st;
        if (opt.timing) {
            HIPCHK(c, hipEventRecord(c->ev[3], s));
            HIPCHK(c, hipEventSynchronize(c->ev[3]));
            ms_table = elapsed(c->ev[2], c->ev[3]);
        }
    }

    // step 3: DD sort of the reference nodes (stable; ties keep grid order)
    if (opt.timing) HIPCHK(c, hipEventRecord(c->ev[4], s));
    if (opt.sort_mode == GAMMAX_SORT_DD && M > 1)
        HIPCHK(c, radix_sort_pairs(c->keys, c->vals, c->tkeys, c->tvals, M, c->hist, s));
    if (opt.timing) HIPCHK(c, hipEventRecord(c->ev[5], s));

    // step 6 (Kernel 3) with step 7 fused: each lane writes gamma at its node index
    if (M > 0) {
        SearchArgs sa{};
        sa.ref = ref;
        sa.ev = ev;
        sa.gamma = gamma;
        sa.order = c->vals;
        sa.guard_list = c->tkeys;   // free after the sort
        sa.sc_in = c->d_sc;
        sa.sc = c->d_sc;
        sa.tab = c->tab;
        sa.tab_len = need_walk ? (int)c->tab_len : 0;
        if (p->ndim == 3) {
            sa.nz = (int)p->shape[0];
            sa.ny = (int)p->shape[1];
            sa.nx = (int)p->shape[2];
        } else {
            sa.nz = 1;
            sa.ny = (int)p->shape[0];
            sa.nx = (int)p->shape[1];
        }
        sa.dd = (float)p->dd;
        sa.dd64 = p->dd;
        sa.local = local ? 1 : 0;
        const int nd = p->ndim;
        const double sx = p->spacing_mm[nd - 1] / p->dta_mm, sy = p->spacing_mm[nd - 2] / p->dta_mm;
        const double sz = nd == 3 ? p->spacing_mm[0] / p->dta_mm : 0.0;
        sa.sx = sx;
        sa.sy = sy;
        sa.sz = sz;
        sa.s2x = (float)(sx * sx);
        sa.s2y = (float)(sy * sy);
        sa.s2z = (float)(sz * sz);
        double smin = std::fmin(sx, sy), smax = std::fmax(sx, sy);
        if (nd == 3) {
            smin = std::fmin(smin, sz);
            smax = std::fmax(smax, sz);
        }
        // kappa(Gram) <= (s_max^2 / s_min^2) * Den for the chain basis of a tetrahedron
        double guard = opt.cond_threshold * (smin * smin) / (smax * smax);
        if (opt.precision != GAMMAX_PREC_GUARDED) guard = INFINITY;
        sa.den_guard = (float)guard;
        HIPCHK(c, launch_search(sa, p->ndim, opt.precision, M, s));
        if (opt.timing) HIPCHK(c, hipEventRecord(c->ev[6], s));
        HIPCHK(c, launch_search_guard(sa, p->ndim, opt.precision, s));
    } else if (opt.timing) {
        HIPCHK(c, hipEventRecord(c->ev[6], s));
    }
    if (opt.timing) HIPCHK(c, hipEventRecord(c->ev[7], s));
    HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));

    const Scalars& h = *c->h_sc;
    res->n_evaluated = h.n_masked;
    res->n_pass = h.n_pass;
    res->n_borderline = h.n_border;
    res->n_fp64_tets = h.n_fp64;
    res->n_cells = h.n_cells;
    res->pass_rate = h.n_masked ? (double)h.n_pass / (double)h.n_masked : NAN;
    res->max_gamma = std::sqrt(u2f(h.maxg2_bits));
    res->dose_max = dmax;
    res->search_radius = std::sqrt(r2);
    res->table_len = need_walk ? (int32_t)c->tab_len : 0;
    if (opt.timing) {
        res->ms_prep = elapsed(c->ev[0], c->ev[1]);
        res->ms_table = ms_table;
        res->ms_sort = elapsed(c->ev[4], c->ev[5]);
        res->ms_search = elapsed(c->ev[5], c->ev[6]);
        res->ms_guard = elapsed(c->ev[6], c->ev[7]);
    }
    return GAMMAX_OK;
}

gammax_status_t gamma_map(const float* ref_dose, const float* eval_dose, int32_t ndim, const int64_t* shape,
                          const double* spacing_mm, double dd, double dta_mm, double dose_threshold,
                          int32_t norm, float* gamma, double* pass_rate, void* stream) {
    static gammax_ctx_t* ctxs[64] = {};
    if (!shape || !spacing_mm || !ref_dose || !eval_dose || !gamma) return GAMMAX_E_NULL;
    if (ndim != 2 && ndim != 3) return GAMMAX_E_SHAPE;
    gammax_problem_t p{};
    p.ndim = ndim;
    p.norm = norm;
    for (int i = 0; i < ndim; ++i) {
        p.shape[i] = shape[i];
        p.spacing_mm[i] = spacing_mm[i];
    }
    p.dd = dd;
    p.dta_mm = dta_mm;
    p.dose_threshold = dose_threshold;
    int64_t n = 0;
    gammax_status_t st = check_problem(nullptr, &p, &n);   // host-side checks before any HIP call
    if (st != GAMMAX_OK) return st;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return GAMMAX_E_DEVICE;
    if (!ctxs[dev]) {
        st = gammax_ctx_create(dev, &ctxs[dev]);
        if (st != GAMMAX_OK) return st;
    }
    gammax_result_t r{};
    st = gammax_map(ctxs[dev], &p, nullptr, ref_dose, eval_dose, gamma, &r, stream);
    if (st == GAMMAX_OK && pass_rate) *pass_rate = r.pass_rate;
    return st;
}

gammax_status_t gammax_sort_pairs(gammax_ctx_t* c, uint32_t* keys, uint32_t* vals, int64_t n, void* stream) {
    if (!c) return GAMMAX_E_NULL;
    if (n < 0) return fail(c, GAMMAX_E_PARAM, "n must be >= 0");
    if (n == 0) return GAMMAX_OK;
    if (!keys || !vals) return fail(c, GAMMAX_E_NULL, "keys and vals are required");
    if (n >= ((int64_t)1 << 31)) return fail(c, GAMMAX_E_PARAM, "n must be < 2^31");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    gammax_status_t st;
    if ((st = grow4(c, &c->keys, &c->vals, &c->tkeys, &c->tvals, &c->item_cap, n)) != GAMMAX_OK) return st;
    if ((st = grow(c, &c->hist, &c->hist_cap, sort_hist_words(n))) != GAMMAX_OK) return st;
    HIPCHK(c, radix_sort_pairs(keys, vals, c->tkeys, c->tvals, n, c->hist, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return GAMMAX_OK;
}

gammax_status_t gammax_build_table(gammax_ctx_t* c, int32_t ndim, const int64_t* shape,
                                   const double* spacing_over_dta, double radius, float* key2_dev,
                                   int32_t* offs_dev, int64_t cap, int64_t* len, void* stream) {
    if (!c) return GAMMAX_E_NULL;
    if (!shape || !spacing_over_dta || !len || !key2_dev || !offs_dev)
        return fail(c, GAMMAX_E_NULL, "shape, spacing, len and output buffers are required");
    if (ndim != 2 && ndim != 3) return fail(c, GAMMAX_E_SHAPE, "ndim must be 2 or 3");
    for (int i = 0; i < ndim; ++i) {
        if (shape[i] < 2 || shape[i] > ((int64_t)1 << 30)) return fail(c, GAMMAX_E_SHAPE, "bad axis length");
        if (!finite_pos(spacing_over_dta[i])) return fail(c, GAMMAX_E_PARAM, "spacing / DTA must be > 0");
    }
    if (!(radius >= 0.0) || !std::isfinite(radius)) return fail(c, GAMMAX_E_PARAM, "radius must be finite, >= 0");
    if (cap < 0) return fail(c, GAMMAX_E_PARAM, "cap must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    *len = 0;
    if (radius == 0.0) return GAMMAX_OK;
    TableGeom g{};
    g.ndim = ndim;
    for (int i = 0; i < 3; ++i) {
        g.shape[i] = i < ndim ? shape[i] : 1;
        g.s[i] = i < ndim ? spacing_over_dta[i] : 1.0;
    }
    g.r2_cap = radius * radius;
    gammax_status_t st = build_table(c, g, s);
    if (st != GAMMAX_OK) return st;
    if (c->tab_len > cap) {
        *len = c->tab_len;
        return fail(c, GAMMAX_E_RADIUS, "table has more entries than cap");
    }
    HIPCHK(c, launch_table_export(c->tab, c->tab_len, ndim, key2_dev, offs_dev, s));
    HIPCHK(c, hipStreamSynchronize(s));
    *len = c->tab_len;
    return GAMMAX_OK;
}

gammax_status_t gammax_pass_count(gammax_ctx_t* c, const float* gamma_dev, int64_t n, uint64_t* counts,
                                  void* stream) {
    if (!c) return GAMMAX_E_NULL;
    if (!gamma_dev || !counts) return fail(c, GAMMAX_E_NULL, "gamma and counts are required");
    if (n < 0) return fail(c, GAMMAX_E_PARAM, "n must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, launch_pass_count(gamma_dev, n, c->d_cnt, s));
    HIPCHK(c, hipMemcpyAsync(c->h_cnt, c->d_cnt, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int i = 0; i < 3; ++i) counts[i] = c->h_cnt[i];
    return GAMMAX_OK;
}

}  // extern "C"
