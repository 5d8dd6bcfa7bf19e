// C ABI of libgammax: argument checks, the per-context workspace and cell-table cache,
// and the device pipeline of one gamma map (Algorithm A2 steps 2-7).
//
// Two ways through a call:
//  * steady state (the cached cell table fits this grid and spacing): every kernel is
//    launched without a host round trip (the masked count M and the radius stay on the
//    device; the grids are sized for all N nodes).  One synchronisation at the end returns
//    the counts.  If the radius turned out larger than the cached table covers, the call
//    is redone below.
//  * table build: the compaction runs first, the host reads M and R, builds the sorted
//    cell table for R (cached with headroom), then queues the search.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gammax.h"
#include "internal.hpp"
#include "model.hpp"

using namespace gammax;

namespace {

// Everything a captured graph depends on; a new capture is made when any of it changes.
struct GraphKey {
    const void* ref;
    const void* ev;
    const void* gamma;
    int32_t ndim, norm;
    int64_t shape[3];
    double spacing[3], dd, dta, thr;
    int32_t sort_mode, precision, tail_lanes, cell_lanes, timing, radius_mode;
    double cond_threshold, radius_factor;
    const void* model;
    int32_t small_sort;
    int32_t short_tail;
    int32_t tail_min_lanes;
    int32_t cnn_pool;
    int32_t projection;
    const float* order_key;
    uint64_t generation;   // bumped on every (re)allocation and table build
};

// A map queued by gammax_map_async: its arguments (for a re-run at collection time), the
// event after the copy of its scalars, and its result if it already ran synchronously.
struct AsyncSlot {
    uint64_t ticket = 0;      // 0: free
    bool done = false;        // ran synchronously; `res` is final
    bool learned = false;
    int ring = -1;            // slot of the pinned scalar ring this map publishes to
    Scalars sc{};             // its scalars, copied out when the ring slot was needed again
    hipEvent_t ev = nullptr;
    hipStream_t stream = nullptr;
    gammax_problem_t p{};
    gammax_options_t o{};
    const float* ref = nullptr;
    const float* eval = nullptr;
    float* gamma = nullptr;
    gammax_result_t res{};
};

}  // namespace

struct gammax_ctx {
    int device = 0;
    std::string err;
    uint64_t generation = 1;
    // per-call scalars
    Scalars* d_sc = nullptr;
    Scalars* h_sc = nullptr;  // pinned
    unsigned long long* d_cnt = nullptr;
    unsigned long long* h_cnt = nullptr;  // pinned
    uint32_t* d_count = nullptr;
    uint32_t* h_count = nullptr;  // pinned (also receives the table's first non-zero key^2)
    // node work lists: 8 arrays of work_cap uint32 in one allocation
    uint32_t* work = nullptr;
    int64_t work_cap = 0;
    uint32_t* blockcnt = nullptr;   // prep tiles: counts, then the tile-group sums
    int64_t blk_cap = 0;
    uint32_t* part = nullptr;       // dose-max partials
    int64_t part_cap = 0;
    uint32_t* hist = nullptr;
    int64_t hist_cap = 0;
    BlockSums* sums = nullptr;
    int64_t sums_cap = 0;
    // cell table cache
    TabEntry* tab = nullptr;
    int64_t tab_cap = 0;
    int64_t tab_len = 0;
    float tab_k1 = INFINITY;        // key^2 of the first row after the zero-key cells
    bool tab_valid = false;
    TableGeom tab_geom{};
    uint32_t* tb = nullptr;         // table build scratch: 4 arrays of tb_cap
    int64_t tb_cap = 0;
    uint32_t* tb_hist = nullptr;
    int64_t tb_hist_cap = 0;
    hipStream_t cap_stream = nullptr;   // private stream on which batch graphs are captured
    bool graph_broken = false;      // a batch graph's capture failed once: batches launch directly
    hipEvent_t ev[12] = {};
    bool events = false;
    // learned radius: features and hidden activations of one grid
    unsigned char* cnn_ws = nullptr;
    int64_t cnn_ws_cap = 0;
    float* yhat = nullptr;          // log(gamma_hat + 0.01) per grid node
    int64_t yhat_cap = 0;
    float* ycoarse = nullptr;       // the network's output on the pooled coarse grid (cnn_pool 2)
    int64_t ycoarse_cap = 0;
    // gammax_map_grids: listed nodes, their first bounds, the guard list (each n_ref words)
    // and the lower-key table of the evaluation grid
    uint32_t* g_work = nullptr;
    int64_t g_work_cap = 0;
    TabEntry* g_tab = nullptr;
    int64_t g_tab_cap = 0, g_tab_len = 0;
    TableGeom g_geom{};
    bool g_tab_valid = false;
    float g_k1 = INFINITY;             // key^2 of its first row past the 27 key-0 cells
    float* g_2d = nullptr;             // 2D two-grid maps: the pair and gamma extruded to two layers
    int64_t g_2d_cap = 0;
    struct BatchState* batch = nullptr;   // gammax_batch state (created on first use)
    struct ManyState* many = nullptr;     // gammax_map_many state (created on first use)
    uint64_t tail_hint = 0;         // tail length of the last map (picks the tail sort variant)
    uint32_t long_rows = 0;         // longest tail walk of the last map, if long (widens the tail groups)
    // maps queued by gammax_map_async and not yet collected
    AsyncSlot* slots = nullptr;     // GAMMAX_ASYNC_SLOTS entries, created on first use
    uint64_t next_ticket = 1;
    // Every map ends with a kernel that writes its scalars into the pinned ring, at the slot
    // given by a device-side map counter, so no runtime copy has to wait for the map's last
    // kernel to drain.  The host counts the maps it launches the same way.
    Scalars* h_ring = nullptr;      // pinned, GAMMAX_ASYNC_SLOTS entries
    uint32_t* d_seq = nullptr;      // device map counter
    uint64_t seq = 0;               // host count of the maps launched
};

void destroy_batch(gammax_ctx* c);

// gammax_map_many: a context per pair index (its table and workspace stay cached
// across calls) and the streams the pairs are spread over: the caller's stream and three
// internal ones (a process gets four hardware queues; a fifth stream would share one).
constexpr int kManyStreams = 4;
struct ManyState {
    std::vector<gammax_ctx*> subs;
    hipStream_t streams[kManyStreams - 1] = {};
    hipEvent_t ev_in = nullptr;
    hipEvent_t ev_out[kManyStreams - 1] = {};
};
void destroy_many(gammax_ctx* c);

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
    "model file cannot be read or written, or is not a model of this network",
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

// Wait for the maps queued by gammax_map_async that may still run (before a buffer or a
// graph that they use is released).
void quiesce(gammax_ctx* c) {
    if (!c->slots) return;
    for (int i = 0; i < GAMMAX_ASYNC_SLOTS; ++i)
        if (c->slots[i].ticket && !c->slots[i].done) (void)hipEventSynchronize(c->slots[i].ev);
}

// The ring slot the next launched map publishes to (the host's count of launched maps;
// the caller adds one once the map is queued).  A queued map that still holds that slot
// has its scalars copied out first.
int claim_ring(gammax_ctx* c) {
    const int r = (int)(c->seq % GAMMAX_ASYNC_SLOTS);
    if (c->slots)
        for (int i = 0; i < GAMMAX_ASYNC_SLOTS; ++i) {
            AsyncSlot& sl = c->slots[i];
            if (sl.ticket && !sl.done && sl.ring == r) {
                (void)hipEventSynchronize(sl.ev);
                sl.sc = c->h_ring[r];
                sl.ring = -1;
            }
        }
    return r;
}

// Grow a device buffer to `need` elements (contents are not kept).
template <typename P>
gammax_status_t grow(gammax_ctx* c, P** p, int64_t* cap, int64_t need) {
    if (need <= *cap && *p) return GAMMAX_OK;
    ++c->generation;
    if (*p) {
        quiesce(c);
        hipError_t e = hipFree(*p);
        *p = nullptr;
        *cap = 0;
        if (e != hipSuccess) return fail(c, GAMMAX_E_DEVICE, std::string("hipFree: ") + hipGetErrorString(e));
    }
    const int64_t n = need > 0 ? need : 1;
    hipError_t e = hipMalloc((void**)p, (size_t)n * sizeof(P));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, GAMMAX_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    *cap = n;
    return GAMMAX_OK;
}

// The node work arrays share one allocation of kWorkArrays * cap words.
enum { W_NODES, W_TAIL_NODE, W_TAIL_F, W_TAIL_KEY, W_TAIL_POS, W_TMP_K, W_TMP_V, W_GUARD, W_FALLBACK, kWorkArrays };
gammax_status_t grow_work(gammax_ctx* c, int64_t n) {
    if (n <= c->work_cap && c->work) return GAMMAX_OK;
    int64_t words = c->work ? kWorkArrays * c->work_cap : 0;
    gammax_status_t st = grow(c, &c->work, &words, kWorkArrays * (n > 0 ? n : 1));
    c->work_cap = st == GAMMAX_OK ? words / kWorkArrays : 0;
    return st;
}
uint32_t* work_array(gammax_ctx* c, int k) { return c->work + (int64_t)k * c->work_cap; }

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
    if (o->sort_mode < GAMMAX_SORT_NONE || o->sort_mode > GAMMAX_SORT_GIVEN)
        return fail(c, GAMMAX_E_PARAM, "unknown sort_mode");
    if (o->sort_mode == GAMMAX_SORT_GIVEN) {
        if (!o->order_key) return fail(c, GAMMAX_E_NULL, "the given order needs order_key");
        if (o->radius_mode != GAMMAX_RADIUS_PLAIN)
            return fail(c, GAMMAX_E_PARAM, "the given order runs with the plain radius only");
    }
    if (o->radius_mode != GAMMAX_RADIUS_PLAIN && o->radius_mode != GAMMAX_RADIUS_LEARNED)
        return fail(c, GAMMAX_E_PARAM, "unknown radius_mode");
    if (!(o->radius_factor >= 1.0) || !std::isfinite(o->radius_factor))
        return fail(c, GAMMAX_E_PARAM, "radius_factor must be finite and >= 1");
    if ((o->radius_mode == GAMMAX_RADIUS_LEARNED || o->sort_mode == GAMMAX_SORT_PREDICTED) && !o->model)
        return fail(c, GAMMAX_E_NULL, "the learned radius and the predicted order need a model");
    if (o->precision < GAMMAX_PREC_FP32 || o->precision > GAMMAX_PREC_FP64)
        return fail(c, GAMMAX_E_PARAM, "unknown precision");
    if (!(o->cond_threshold >= 1.0)) return fail(c, GAMMAX_E_PARAM, "cond_threshold must be >= 1");
    if (o->timing != 0 && o->timing != 1) return fail(c, GAMMAX_E_PARAM, "timing must be 0 or 1");
    const int tl = o->tail_lanes;
    if (!(tl == 0 || tl == 1 || tl == 8 || tl == 16 || tl == 32 || tl == 64))
        return fail(c, GAMMAX_E_PARAM, "tail_lanes must be 0, 1, 8, 16, 32 or 64");
    if (!(o->cell_lanes == 0 || o->cell_lanes == 1 || o->cell_lanes == 4 || o->cell_lanes == 8))
        return fail(c, GAMMAX_E_PARAM, "cell_lanes must be 0, 1, 4 or 8");
    if (o->autotune != 0 && o->autotune != 1) return fail(c, GAMMAX_E_PARAM, "autotune must be 0 or 1");
    if (o->cnn_pool != 0 && o->cnn_pool != 2) return fail(c, GAMMAX_E_PARAM, "cnn_pool must be 0 or 2");
    if (o->projection != 0 && o->projection != 1) return fail(c, GAMMAX_E_PARAM, "projection must be 0 or 1");
    for (int i = 0; i < 1; ++i)
        if (o->reserved[i] != 0) return fail(c, GAMMAX_E_PARAM, "reserved option fields must be 0");
    if (o->model && c && o->model->device != c->device)
        return fail(c, GAMMAX_E_PARAM, "model and context live on different devices");
    return GAMMAX_OK;
}

__global__ void k_zero_u32(uint32_t* p) {
    if (threadIdx.x == 0) *p = 0u;
}

// The map's scalars into the pinned ring at the slot of the device map counter, made
// visible at system scope before the kernel ends; then the counter moves on.  One wave:
// every lane reads the same counter value.  (A runtime device-to-host copy queued after the
// map's last kernel starts several microseconds after it; a kernel follows at once.)
__device__ __forceinline__ void publish_body(const Scalars* __restrict__ src, uint32_t* seq, Scalars* ring) {
    constexpr int W = (int)(sizeof(Scalars) / sizeof(uint32_t));
    static_assert(sizeof(Scalars) % sizeof(uint32_t) == 0, "Scalars is a whole number of words");
    const uint32_t k = *seq;
    Scalars* dst = ring + (k % GAMMAX_ASYNC_SLOTS);
    const int t = threadIdx.x;
    if (t < W) reinterpret_cast<volatile uint32_t*>(dst)[t] = reinterpret_cast<const uint32_t*>(src)[t];
    if (t == 0) *seq = k + 1u;
    __threadfence_system();
}
__global__ void k_publish_scalars(const Scalars* __restrict__ src, uint32_t* seq, Scalars* ring) {
    publish_body(src, seq, ring);
}
// Every pair of a batch publishes its scalars (block i: pair i).
__global__ void k_batch_publish(const BatchPair* __restrict__ pairs) {
    const BatchPair& P = pairs[blockIdx.x];
    publish_body(P.sa.sc, P.seq, P.ring);
}

bool same_geom(const TableGeom& a, const TableGeom& b) {
    if (a.ndim != b.ndim || a.lower != b.lower) return false;
    for (int i = 0; i < a.ndim; ++i)
        if (a.shape[i] != b.shape[i] || a.s[i] != b.s[i]) return false;
    return true;
}

float round_down_float(double x) {
    float f = (float)x;
    if ((double)f > x) f = std::nextafter(f, -INFINITY);
    return f;
}

// Build the sorted cell table for `g` into *tab (grown as needed; synchronises `s`).
// *len receives the row count, *k1 the key^2 of the first row after the 2^d key-0 rows.
gammax_status_t build_rows(gammax_ctx* c, TableGeom& g, TabEntry** tab, int64_t* cap, int64_t* len, float* k1,
                           hipStream_t s) {
    table_box(g);
    if (g.box > kMaxTableBox)
        return fail(c, GAMMAX_E_RADIUS, "cell table candidate box of " + std::to_string(g.box) + " entries");
    ++c->generation;
    gammax_status_t st;
    if (g.box > c->tb_cap || !c->tb) {
        int64_t words = c->tb ? 4 * c->tb_cap : 0;
        c->tb_cap = 0;
        if ((st = grow(c, &c->tb, &words, 4 * g.box)) != GAMMAX_OK) return st;
        c->tb_cap = words / 4;
    }
    if ((st = grow(c, &c->tb_hist, &c->tb_hist_cap, sort_hist_words(g.box))) != GAMMAX_OK) return st;
    uint32_t* keys = c->tb;
    uint32_t* vals = c->tb + c->tb_cap;
    uint32_t* tk = c->tb + 2 * c->tb_cap;
    uint32_t* tv = c->tb + 3 * c->tb_cap;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, c->d_count);
    HIPCHK(c, launch_table_gen(g, keys, vals, c->d_count, s));
    HIPCHK(c, radix_sort_pairs(keys, vals, tk, tv, g.box, nullptr, c->tb_hist, s));
    HIPCHK(c, hipMemcpyAsync(c->h_count, c->d_count, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const int64_t T = *c->h_count;
    if ((st = grow(c, tab, cap, T)) != GAMMAX_OK) return st;
    HIPCHK(c, launch_table_rows(g, vals, T, *tab, s));
    const int zero_rows = g.lower ? 27 : (g.ndim == 3 ? 8 : 4);
    *k1 = INFINITY;
    if (T > zero_rows) {
        HIPCHK(c, hipMemcpyAsync(c->h_count, &(*tab)[zero_rows].key2, sizeof(float), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        std::memcpy(k1, c->h_count, sizeof(float));
    }
    *len = T;
    return GAMMAX_OK;
}

// Build the context's own table (the single-pair path) for `g`.
gammax_status_t build_table(gammax_ctx* c, TableGeom g, hipStream_t s) {
    c->tab_valid = false;
    gammax_status_t st = build_rows(c, g, &c->tab, &c->tab_cap, &c->tab_len, &c->tab_k1, s);
    if (st != GAMMAX_OK) return st;
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
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();   // do not leave an ignored error for the caller's next check
        return 0.0f;
    }
    return ms;
}

struct CallSetup {
    const gammax_problem_t* p;
    const gammax_options_t* opt;
    const float* ref;
    const float* ev;
    float* gamma;
    int64_t n;
};

// Workspace of the CNN over one grid: features (o+8, 2 channels), then the hidden
// activations of layers 2 and 3 (o+4, o+2; 16 channels), each 256-byte aligned.  Layer 1's
// output (o+6) is never stored: layers 1 and 2 run fused.
struct CnnWs {
    uint16_t *feat, *a2, *a3;
    int64_t bytes;
};
CnnWs cnn_layout(unsigned char* base, const int o[3]) {
    CnnWs w{};
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        uint16_t* p = base ? (uint16_t*)(base + off) : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    int sh[3];
    act_shape(o, 8, sh);
    w.feat = take(vol_of(sh) * 4);
    act_shape(o, 4, sh);
    w.a2 = take(vol_of(sh) * 32);
    act_shape(o, 2, sh);
    w.a3 = take(vol_of(sh) * 32);
    w.bytes = off;
    return w;
}

gammax_status_t grow_cnn(gammax_ctx* c, const int o[3], CnnWs* w) {
    const int64_t need = cnn_layout(nullptr, o).bytes;
    if (need > c->cnn_ws_cap || !c->cnn_ws) {
        gammax_status_t st = grow(c, &c->cnn_ws, &c->cnn_ws_cap, need);
        if (st != GAMMAX_OK) return st;
    }
    *w = cnn_layout(c->cnn_ws, o);
    return GAMMAX_OK;
}

// Workspace of the pooled network input (cnn_pool 2) of a 3D problem: the CNN workspace of
// the coarse grid and its output.
gammax_status_t grow_pooled(gammax_ctx* c, const gammax_problem_t* p) {
    const int n[3] = {(int)p->shape[0], (int)p->shape[1], (int)p->shape[2]};
    int co[3];
    pool2_shape(n, co);
    CnnWs w;
    gammax_status_t st = grow_cnn(c, co, &w);
    if (st != GAMMAX_OK) return st;
    return grow(c, &c->ycoarse, &c->ycoarse_cap, (int64_t)co[0] * co[1] * co[2]);
}

// The model is used on 3D problems when the learned radius or the predicted order is asked
// for (2D problems keep the plain radius and order by |DD|).
bool uses_model(const gammax_problem_t* p, const gammax_options_t* o) {
    return p->ndim == 3 && o->model &&
           (o->radius_mode == GAMMAX_RADIUS_LEARNED || o->sort_mode == GAMMAX_SORT_PREDICTED);
}

// A short tail (the previous map's held at most SMALL_SORT_CAP nodes) in the automatic
// layout walks in groups of 64 lanes, where a walk of under 64 rows is one batch whatever
// its bound: the learned radius's speculative bound cannot shorten it, and a fallback would
// add a batch and a launch.  Such a tail walks with the plain bound (the same result); the
// nodes the prediction would not have certified are still counted.
bool short_tail(const gammax_ctx* c, const gammax_options_t& opt) {
    return opt.tail_lanes == 0 && c->tail_hint <= (uint64_t)SMALL_SORT_CAP;
}

// Least lanes per node of the automatic tail layout: wide enough that the longest walk of
// the context's last map (if it was long) takes about 32 dependent steps.
int tail_min_lanes(const gammax_ctx* c) {
    if (c->long_rows == 0) return 0;
    int g = 8;
    while (g < 64 && (uint64_t)g * 32 < c->long_rows) g <<= 1;
    return g;
}

// Queue the compaction (Kernel 1).  ev0/ev1 (optional) bracket it.
// Compaction arguments of one map on the context's workspace.
PrepArgs make_prep_args(gammax_ctx* c, const CallSetup& cs) {
    const int64_t ntiles = prep_tiles(cs.n);
    PrepArgs pa{};
    pa.ref = cs.ref;
    pa.ev = cs.ev;
    pa.gamma = cs.gamma;
    pa.n = cs.n;
    pa.thr = (float)cs.p->dose_threshold;
    pa.dd = (float)cs.p->dd;
    pa.local = cs.p->norm == GAMMAX_LOCAL ? 1 : 0;
    pa.sc = c->d_sc;
    pa.part = c->part;
    pa.blockcnt = c->blockcnt;
    prep_groups(cs.n, &pa.super_shift, &pa.n_super);
    pa.super = c->blockcnt + ntiles;
    pa.ntiles = (int)ntiles;
    pa.nodes = work_array(c, W_NODES);
    pa.sums = c->sums;
    pa.mbits = reinterpret_cast<unsigned long long*>(c->blockcnt + prep_mbits_offset(cs.n));
    return pa;
}

gammax_status_t enqueue_prep(gammax_ctx* c, const CallSetup& cs, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (ev0) HIPCHK(c, hipEventRecord(ev0, s));
    const PrepArgs pa = make_prep_args(c, cs);
    HIPCHK(c, launch_prep(pa, s));
    if (ev1) HIPCHK(c, hipEventRecord(ev1, s));
    return GAMMAX_OK;
}

// The network at the nodes queued for the tail walk, queued right after the key-0 pass:
// y per tail item into `y` and, for the predicted order, the sort keys.
struct TailCnnHook {
    const gammax_model* model;
    const float* ref;
    const float* ev;
    int shape[3];
    // cnn_pool 2: the pooled pair's features, coarse activations and output
    bool pooled;
    CnnWs ws;
    float* ycoarse;
    const Scalars* sc;
    const uint32_t* nodes;
    const uint32_t* count;
    float* y;
    uint32_t* key;
    hipEvent_t ev0, ev1;     // optional timing
    int blocks;
};

// The given order: the caller's key of every queued tail node, written where the network
// writes its predictions in the predicted order.
struct GivenKeyHook {
    const uint32_t* nodes;
    const uint32_t* count;
    const float* given;
    uint32_t* key;
};

hipError_t given_key_hook(void* user, hipStream_t s) {
    const GivenKeyHook& h = *static_cast<const GivenKeyHook*>(user);
    return launch_given_keys(h.nodes, h.count, h.given, h.key, s);
}

hipError_t tail_cnn_hook(void* user, hipStream_t s) {
    const TailCnnHook& h = *static_cast<const TailCnnHook*>(user);
    hipError_t e;
    if (h.ev0 && (e = hipEventRecord(h.ev0, s)) != hipSuccess) return e;
    gammax_model* m = const_cast<gammax_model*>(h.model);
    if (h.pooled) {
        int co[3];
        pool2_shape(h.shape, co);
        if ((e = launch_features_pool2(h.ref, h.ev, h.shape, h.sc, h.ws.feat, s)) != hipSuccess) return e;
        if ((e = model_forward(m, h.ws.feat, 1, co, nullptr, h.ws.a2, h.ws.a3, h.ycoarse, s)) != hipSuccess) return e;
        if ((e = launch_cnn_upsample(h.ycoarse, h.shape, h.nodes, h.count, h.blocks, h.y, h.key, s)) != hipSuccess)
            return e;
        if (h.ev1 && (e = hipEventRecord(h.ev1, s)) != hipSuccess) return e;
        return hipSuccess;
    }
    const uint16_t* frag[3] = {frag_fwd(m, 0), frag_fwd(m, 1), frag_fwd(m, 2)};
    const float* bias[3] = {layer_bias(m, 0), layer_bias(m, 1), layer_bias(m, 2)};
    e = launch_cnn_tail(h.ref, h.ev, h.shape, h.sc, h.nodes, h.count, h.blocks, frag, bias, m->theta + CNN_OFF[3],
                        layer_bias(m, 3), h.y, h.key, s);
    if (e != hipSuccess) return e;
    if (h.ev1 && (e = hipEventRecord(h.ev1, s)) != hipSuccess) return e;
    return hipSuccess;
}

// Point the hook at the pooled workspace (sized by grow_pooled for this problem).
void set_pooled(gammax_ctx* c, TailCnnHook* h) {
    int co[3];
    pool2_shape(h->shape, co);
    h->pooled = true;
    h->ws = cnn_layout(c->cnn_ws, co);
    h->ycoarse = c->ycoarse;
}

constexpr int kTailCnnBlocks = 2048;   // grid-stride one-wave blocks of the network at the tail nodes (8 per CU)

// Search arguments of one pair.  work: the kWorkArrays node arrays, `stride` words apart.
SearchArgs make_search_args(const gammax_problem_t* p, const gammax_options_t& opt, const float* ref,
                            const float* ev, float* gamma, Scalars* sc, const TabEntry* tab, int tab_len, float k1,
                            float r2_cap, uint32_t* work, int64_t stride, BlockSums* sums, const float* yhat) {
    SearchArgs sa{};
    sa.ref = ref;
    sa.ev = ev;
    sa.gamma = gamma;
    sa.sc = sc;
    sa.tab = tab;
    sa.tab_len = tab_len;
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
    sa.local = p->norm == GAMMAX_LOCAL ? 1 : 0;
    const int nd = p->ndim;
    const double sx = p->spacing_mm[nd - 1] / p->dta_mm, sy = p->spacing_mm[nd - 2] / p->dta_mm;
    const double sz = nd == 3 ? p->spacing_mm[0] / p->dta_mm : 0.0;
    sa.sx = sx;
    sa.sy = sy;
    sa.sz = sz;
    sa.s2x = (float)(sx * sx);
    sa.s2y = (float)(sy * sy);
    sa.s2z = (float)(sz * sz);
    {
        // FP32 divisions, as the kernels would form them (IEEE round to nearest)
        const float x2 = sa.s2x, y2 = sa.s2y, z2 = sa.s2z;
        sa.inv_s2[0] = 1.0f / x2;
        sa.inv_s2[1] = 1.0f / y2;
        sa.inv_s2[2] = z2 > 0.0f ? 1.0f / z2 : 0.0f;
        sa.inv_s2[3] = 1.0f / (x2 + y2);
        sa.inv_s2[4] = z2 > 0.0f ? 1.0f / (x2 + z2) : 0.0f;
        sa.inv_s2[5] = z2 > 0.0f ? 1.0f / (y2 + z2) : 0.0f;
        sa.inv_s2[6] = 1.0f / ((x2 + y2) + z2);
    }
    double smin = std::fmin(sx, sy), smax = std::fmax(sx, sy);
    if (nd == 3) {
        smin = std::fmin(smin, sz);
        smax = std::fmax(smax, sz);
    }
    // kappa(Gram) <= (s_max^2 / s_min^2) * Den for the chain basis of a tetrahedron
    double guard = opt.cond_threshold * (smin * smin) / (smax * smax);
    if (opt.precision != GAMMAX_PREC_GUARDED) guard = INFINITY;
    sa.den_guard = (float)guard;
    sa.k1 = k1;
    sa.r2_cap = r2_cap;
    const bool learned = uses_model(p, &opt);
    sa.tail_key = opt.sort_mode == GAMMAX_SORT_BOUND
                      ? 1
                      : (((opt.sort_mode == GAMMAX_SORT_PREDICTED && learned) || opt.sort_mode == GAMMAX_SORT_GIVEN) ? 2 : 0);
    sa.yhat = learned ? yhat : nullptr;
    sa.spec_factor = (float)opt.radius_factor;
    sa.fb_list = work + W_FALLBACK * stride;
    sa.nodes = work + W_NODES * stride;
    sa.tail_node = work + W_TAIL_NODE * stride;
    sa.tail_f = work + W_TAIL_F * stride;
    sa.tail_key_arr = work + W_TAIL_KEY * stride;
    sa.tail_pos = work + W_TAIL_POS * stride;
    sa.guard_list = work + W_GUARD * stride;
    sa.sums = sums;
    return sa;
}

// The 2^d zero-key cells of a problem in table order: offsets in {-1,0}^d, slowest first.
ZeroGeo make_zero_geo(const gammax_problem_t* p) {
    ZeroGeo z{};
    const int nd = p->ndim;
    const double s3[3] = {p->spacing_mm[0] / p->dta_mm, p->spacing_mm[1] / p->dta_mm,
                          nd == 3 ? p->spacing_mm[2] / p->dta_mm : 1.0};
    for (int k = 0; k < (nd == 3 ? 8 : 4); ++k) {
        if (nd == 3) table_row_host(3, s3, (k >> 2) - 1, ((k >> 1) & 1) - 1, (k & 1) - 1, &z.row[k]);
        else table_row_host(2, s3, 0, (k >> 1) - 1, (k & 1) - 1, &z.row[k]);
    }
    return z;
}

// Queue the search (steps 3, 6, 7) over at most m_bound nodes with the cached table.
gammax_status_t enqueue_search(gammax_ctx* c, const CallSetup& cs, uint32_t m_bound, float r2_cap,
                               hipStream_t s, bool timing, bool skip_zero = false) {
    const gammax_problem_t* p = cs.p;
    const gammax_options_t& opt = *cs.opt;
    const SearchArgs sa = make_search_args(p, opt, cs.ref, cs.ev, cs.gamma, c->d_sc, c->tab,
                                           c->tab_valid ? (int)c->tab_len : 0, c->tab_valid ? c->tab_k1 : INFINITY,
                                           r2_cap, c->work, c->work_cap, c->sums, c->yhat);
    const bool learned = uses_model(p, &opt);
    SearchPlan plan{};
    plan.ndim = p->ndim;
    plan.precision = opt.precision;
    plan.tail_lanes = opt.tail_lanes;
    plan.tail_min_lanes = tail_min_lanes(c);
    // one lane per node (shared neighbourhood loads) unless one lane per cell is asked for
    plan.zero_lanes = (opt.cell_lanes == 4 || opt.cell_lanes == 8) ? 1 : 0;
    plan.projection = opt.projection;
    plan.skip_zero = skip_zero ? 1 : 0;
    plan.spec = (learned && opt.radius_mode == GAMMAX_RADIUS_LEARNED) ? (short_tail(c, opt) ? 3 : 1) : 0;
    plan.M = m_bound;
    plan.zero = make_zero_geo(p);
    plan.tmp_keys = work_array(c, W_TMP_K);
    plan.tmp_vals = work_array(c, W_TMP_V);
    plan.hist = opt.sort_mode == GAMMAX_SORT_NONE ? nullptr : c->hist;
    plan.small_sort = c->tail_hint <= (uint64_t)SMALL_SORT_CAP ? 1 : 0;
    TailCnnHook hook{};
    if (learned) {
        hook.model = opt.model;
        hook.ref = cs.ref;
        hook.ev = cs.ev;
        for (int i = 0; i < 3; ++i) hook.shape[i] = (int)p->shape[i];
        hook.sc = c->d_sc;
        hook.nodes = work_array(c, W_TAIL_NODE);
        hook.count = &c->d_sc->n_tail;
        hook.y = c->yhat;
        hook.key = sa.tail_key == 2 ? work_array(c, W_TAIL_KEY) : nullptr;
        hook.ev0 = timing ? c->ev[9] : nullptr;
        hook.ev1 = timing ? c->ev[10] : nullptr;
        hook.blocks = kTailCnnBlocks;
        if (opt.cnn_pool == 2) set_pooled(c, &hook);
        plan.after_zero = tail_cnn_hook;
        plan.after_zero_user = &hook;
    }
    GivenKeyHook ghook{};
    if (opt.sort_mode == GAMMAX_SORT_GIVEN) {
        ghook.nodes = work_array(c, W_TAIL_NODE);
        ghook.count = &c->d_sc->n_tail;
        ghook.given = opt.order_key;
        ghook.key = work_array(c, W_TAIL_KEY);
        plan.after_zero = given_key_hook;
        plan.after_zero_user = &ghook;
    }
    if (timing) {
        HIPCHK(c, hipEventRecord(c->ev[4], s));
        plan.ev_shell_end = c->ev[5];
        plan.ev_sort_end = c->ev[6];
        plan.ev_tail_end = c->ev[7];
    }
    HIPCHK(c, launch_search(sa, plan, s));
    if (timing) HIPCHK(c, hipEventRecord(c->ev[8], s));
    hipLaunchKernelGGL(k_publish_scalars, dim3(1), dim3(64), 0, s, (const Scalars*)c->d_sc, c->d_seq, c->h_ring);
    HIPCHK(c, hipGetLastError());
    return GAMMAX_OK;
}

GraphKey key_of(gammax_ctx* c, const CallSetup& cs) {
    GraphKey k;
    std::memset(&k, 0, sizeof(k));
    k.ref = cs.ref;
    k.ev = cs.ev;
    k.gamma = cs.gamma;
    k.ndim = cs.p->ndim;
    k.norm = cs.p->norm;
    for (int i = 0; i < 3; ++i) {
        k.shape[i] = i < cs.p->ndim ? cs.p->shape[i] : 0;
        k.spacing[i] = i < cs.p->ndim ? cs.p->spacing_mm[i] : 0.0;
    }
    k.dd = cs.p->dd;
    k.dta = cs.p->dta_mm;
    k.thr = cs.p->dose_threshold;
    k.sort_mode = cs.opt->sort_mode;
    k.precision = cs.opt->precision;
    k.tail_lanes = cs.opt->tail_lanes;
    k.cell_lanes = cs.opt->cell_lanes;
    k.timing = cs.opt->timing;
    k.radius_mode = cs.opt->radius_mode;
    k.cond_threshold = cs.opt->cond_threshold;
    k.radius_factor = cs.opt->radius_factor;
    k.model = cs.opt->model;
    k.small_sort = (cs.opt->sort_mode != GAMMAX_SORT_NONE && c->tail_hint <= (uint64_t)SMALL_SORT_CAP) ? 1 : 0;
    k.short_tail = short_tail(c, *cs.opt) ? 1 : 0;
    k.tail_min_lanes = tail_min_lanes(c);
    k.cnn_pool = cs.opt->cnn_pool;
    k.projection = cs.opt->projection;
    k.order_key = cs.opt->sort_mode == GAMMAX_SORT_GIVEN ? cs.opt->order_key : nullptr;
    k.generation = c->generation;
    return k;
}

void fill_result_from(gammax_ctx* c, const Scalars& h, gammax_result_t* res, bool timing, float ms_table,
                      bool cnn) {
    const float r2 = u2f(h.r2_bits);
    res->n_evaluated = h.n_masked;
    res->n_pass = h.n_pass;
    res->n_borderline = h.n_border;
    res->n_fp64_tets = h.n_fp64;
    res->n_cells = h.n_cells;
    res->n_tail = h.n_tail;
    res->n_guarded = h.n_guard;
    res->pass_rate = h.n_masked ? (double)h.n_pass / (double)h.n_masked : NAN;
    res->max_gamma = std::sqrt(u2f(h.maxg2_bits));
    res->dose_max = ord_to_float(h.dmax_ord);
    res->search_radius = std::sqrt(r2);
    res->table_len = (h.n_masked > 0 && r2 > 0.0f) ? (int32_t)c->tab_len : 0;
    if (timing) {
        res->ms_prep = elapsed(c->ev[0], c->ev[1]);
        res->ms_table = ms_table;
        res->ms_search = elapsed(c->ev[4], c->ev[5]);
        // with the learned radius the network at the tail nodes runs between the key-0 pass
        // and the sort (ms_cnn)
        res->ms_sort = cnn ? elapsed(c->ev[10], c->ev[6]) : elapsed(c->ev[5], c->ev[6]);
        res->ms_tail = elapsed(c->ev[6], c->ev[7]);
        res->ms_guard = elapsed(c->ev[7], c->ev[8]);
        res->ms_cnn = cnn ? elapsed(c->ev[9], c->ev[10]) : 0.0f;
    }
    res->n_fallback = (uint64_t)h.n_fallback + h.n_fallback_inline;
    res->long_walk_rows = h.long_rows;
    // the next call sorts its tail with the rank sort if this one's would have fitted, and
    // widens its tail groups if this one had long walks
    c->tail_hint = h.sort_overflow ? (uint64_t)SMALL_SORT_CAP + 1 : h.n_tail;
    c->long_rows = h.long_rows;
}

void fill_result(gammax_ctx* c, gammax_result_t* res, bool timing, float ms_table, bool cnn) {
    fill_result_from(c, *c->h_sc, res, timing, ms_table, cnn);
}

gammax_status_t scalar_errors(gammax_ctx* c, const Scalars& h, bool local) {
    if (h.flags & FLAG_NONFINITE) return fail(c, GAMMAX_E_NONFINITE, "a dose value is NaN or infinite");
    if (!local && !(ord_to_float(h.dmax_ord) > 0.0f))
        return fail(c, GAMMAX_E_DOSE, "max reference dose is not positive");
    return GAMMAX_OK;
}

gammax_status_t device_errors(gammax_ctx* c, bool local) { return scalar_errors(c, *c->h_sc, local); }

// Dose maximum and the global 1/dD of a pair into the context's scalars.
gammax_status_t enqueue_dose_scalars(gammax_ctx* c, const gammax_problem_t* p, const float* ref, const float* ev,
                                     int64_t n, hipStream_t s) {
    gammax_status_t st = grow(c, &c->part, &c->part_cap, 2 * MAX_BLOCKS);
    if (st != GAMMAX_OK) return st;
    PrepArgs pa{};
    pa.ref = ref;
    pa.ev = ev;
    pa.n = n;
    pa.thr = (float)p->dose_threshold;
    pa.dd = (float)p->dd;
    pa.local = p->norm == GAMMAX_LOCAL ? 1 : 0;
    pa.sc = c->d_sc;
    pa.part = c->part;
    HIPCHK(c, launch_dose_scalars(pa, s));
    return GAMMAX_OK;
}

gammax_status_t model_inputs(gammax_ctx* c, const gammax_problem_t* p, const float* ref, const float* ev,
                             int o[3], int64_t* n) {
    if (!ref || !ev) return fail(c, GAMMAX_E_NULL, "dose pointers are required");
    gammax_status_t st = check_problem(c, p, n);
    if (st != GAMMAX_OK) return st;
    if (p->ndim != 3) return fail(c, GAMMAX_E_SHAPE, "the learned radius is 3D only");
    for (int i = 0; i < 3; ++i) o[i] = (int)p->shape[i];
    return GAMMAX_OK;
}

// Checks and workspace of one map call (every step of the steady path then runs without a
// host round trip).  *opt receives the options in effect, *n the node count.
gammax_status_t map_setup(gammax_ctx* c, const gammax_problem_t* p, const gammax_options_t* opt_in,
                          const float* ref, const float* ev, const float* gamma, gammax_options_t* opt,
                          int64_t* n, bool* learned) {
    if (!ref || !ev || !gamma) return fail(c, GAMMAX_E_NULL, "dose and gamma pointers are required");
    gammax_status_t st = check_problem(c, p, n);
    if (st != GAMMAX_OK) return st;
    if (gamma == ref || gamma == ev) return fail(c, GAMMAX_E_PARAM, "gamma must not alias the dose arrays");
    if (opt_in) *opt = *opt_in;
    else gammax_options_default(opt);
    if ((st = check_options(c, opt)) != GAMMAX_OK) return st;
    HIPCHK(c, hipSetDevice(c->device));
    // workspace, sized for all n nodes so that the steady path needs no count from the host
    if ((st = grow_work(c, *n)) != GAMMAX_OK) return st;
    if ((st = grow(c, &c->blockcnt, &c->blk_cap, prep_words(*n))) != GAMMAX_OK) return st;
    if ((st = grow(c, &c->part, &c->part_cap, 2 * MAX_BLOCKS)) != GAMMAX_OK) return st;
    if ((st = grow(c, &c->hist, &c->hist_cap, sort_hist_words(*n))) != GAMMAX_OK) return st;
    if ((st = grow(c, &c->sums, &c->sums_cap, search_sums_needed((uint32_t)*n))) != GAMMAX_OK) return st;
    if (opt->timing && (st = ensure_events(c)) != GAMMAX_OK) return st;
    *learned = uses_model(p, opt);
    if (*learned && (st = grow(c, &c->yhat, &c->yhat_cap, *n)) != GAMMAX_OK) return st;
    if (*learned && opt->cnn_pool == 2 && (st = grow_pooled(c, p)) != GAMMAX_OK) return st;
    return GAMMAX_OK;
}

bool steady_table(const gammax_ctx* c, const gammax_problem_t* p) {
    return c->tab_valid && same_geom(c->tab_geom, geom_of(p));
}

// The whole map on the cached table, its kernels launched directly on the caller's stream.
// (Replaying the same seven kernels from a captured HIP graph was measured slower on this
// stack: 0.0894 against 0.0840 ms per queued map at 128x128x96, 0.078 against 0.064 ms per
// map with 16 maps on four streams.)
gammax_status_t enqueue_steady(gammax_ctx* c, const CallSetup& cs, bool timing, hipStream_t s) {
    gammax_status_t st;
    const uint32_t n = (uint32_t)cs.n;
    const float r2_cap = round_down_float(c->tab_geom.r2_cap);
    if ((st = enqueue_prep(c, cs, s, timing ? c->ev[0] : nullptr, timing ? c->ev[1] : nullptr)) != GAMMAX_OK)
        return st;
    return enqueue_search(c, cs, n, r2_cap, s, timing);
}

}  // namespace

extern "C" {

void gammax_options_default(gammax_options_t* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->sort_mode = GAMMAX_SORT_NONE;
    opt->precision = GAMMAX_PREC_GUARDED;
    opt->cond_threshold = 1e6;
    opt->timing = 0;
    opt->tail_lanes = 0;
    opt->radius_mode = GAMMAX_RADIUS_PLAIN;
    opt->model = nullptr;
    opt->radius_factor = 1.1;
}

const char* gammax_status_string(gammax_status_t st) {
    const int k = -(int)st;
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
        hipHostMalloc((void**)&c->h_count, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_ring, sizeof(Scalars) * GAMMAX_ASYNC_SLOTS, hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&c->d_seq, sizeof(uint32_t)) != hipSuccess ||
        hipMemset(c->d_seq, 0, sizeof(uint32_t)) != hipSuccess) {
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
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    void* dev[] = {c->d_sc, c->d_cnt, c->d_count, c->d_seq, c->work, c->blockcnt, c->part, c->hist,
                   c->sums, c->tab, c->tb, c->tb_hist, c->cnn_ws, c->yhat, c->ycoarse, c->g_work, c->g_tab,
                   c->g_2d};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    destroy_batch(c);
    destroy_many(c);
    if (c->slots) {
        for (int i = 0; i < GAMMAX_ASYNC_SLOTS; ++i) (void)hipEventDestroy(c->slots[i].ev);
        delete[] c->slots;
    }
    void* host[] = {c->h_sc, c->h_cnt, c->h_count, c->h_ring};
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
    if (!res) return fail(c, GAMMAX_E_NULL, "result pointer is required");
    int64_t n = 0;
    bool learned = false;
    gammax_options_t opt;
    gammax_status_t st = map_setup(c, p, opt_in, ref, ev, gamma, &opt, &n, &learned);
    if (st != GAMMAX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    std::memset(res, 0, sizeof(*res));
    const bool timing = opt.timing != 0;
    const bool local = p->norm == GAMMAX_LOCAL;
    CallSetup cs{p, &opt, ref, ev, gamma, n};
    const TableGeom g = geom_of(p);

    // steady state: the cached table serves this geometry; no host round trip before the end
    if (steady_table(c, p)) {
        const int r = claim_ring(c);
        if ((st = enqueue_steady(c, cs, timing, s)) != GAMMAX_OK) return st;
        ++c->seq;
        HIPCHK(c, hipStreamSynchronize(s));
        *c->h_sc = c->h_ring[r];
        if ((st = device_errors(c, local)) != GAMMAX_OK) return st;
        if (!(c->h_sc->flags & FLAG_TABLE_SHORT)) {
            fill_result(c, res, timing, 0.0f, learned);
            return GAMMAX_OK;
        }
        // the radius outgrew the cached table: build a larger one below and run again
    }

    // table build: compaction first, then the table for the radius found, then the search
    if ((st = enqueue_prep(c, cs, s, timing ? c->ev[0] : nullptr, timing ? c->ev[1] : nullptr)) != GAMMAX_OK)
        return st;
    HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    if ((st = device_errors(c, local)) != GAMMAX_OK) return st;
    const uint32_t M = c->h_sc->n_masked;
    const float r2 = u2f(c->h_sc->r2_bits);
    float ms_table = 0.0f;
    if (M > 0 && r2 > 0.0f) {
        TableGeom gb = g;
        gb.r2_cap = (double)r2 * 1.5;   // headroom so that nearby radii reuse the table
        if (timing) HIPCHK(c, hipEventRecord(c->ev[2], s));
        if ((st = build_table(c, gb, s)) != GAMMAX_OK) return st;
        if (timing) {
            HIPCHK(c, hipEventRecord(c->ev[3], s));
            HIPCHK(c, hipEventSynchronize(c->ev[3]));
            ms_table = elapsed(c->ev[2], c->ev[3]);
        }
    }
    if (M > 0) {
        const bool walk = r2 > 0.0f && c->tab_valid;
        const bool keep = c->tab_valid;
        if (!walk) c->tab_valid = false;   // no table needed (every gamma0 is 0)
        const int r = claim_ring(c);
        st = enqueue_search(c, cs, M, INFINITY, s, timing);
        c->tab_valid = keep;
        if (st != GAMMAX_OK) return st;
        ++c->seq;
        HIPCHK(c, hipStreamSynchronize(s));
        *c->h_sc = c->h_ring[r];
    } else {
        if (timing)
            for (int k = 4; k <= 10; ++k) HIPCHK(c, hipEventRecord(c->ev[k], s));
        HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    fill_result(c, res, timing, ms_table, learned);
    return GAMMAX_OK;
}

gammax_status_t gammax_map_async(gammax_ctx_t* c, const gammax_problem_t* p, const gammax_options_t* opt_in,
                                 const float* ref, const float* ev, float* gamma, uint64_t* ticket, void* stream) {
    if (!c) return GAMMAX_E_NULL;
    if (!ticket) return fail(c, GAMMAX_E_NULL, "ticket pointer is required");
    *ticket = 0;
    if (opt_in && opt_in->timing) return fail(c, GAMMAX_E_PARAM, "timing is not available for queued maps");
    int64_t n = 0;
    bool learned = false;
    gammax_options_t opt;
    gammax_status_t st = map_setup(c, p, opt_in, ref, ev, gamma, &opt, &n, &learned);
    if (st != GAMMAX_OK) return st;
    if (!c->slots) {
        AsyncSlot* sl = new (std::nothrow) AsyncSlot[GAMMAX_ASYNC_SLOTS];
        if (!sl) return fail(c, GAMMAX_E_NOMEM, "queued map slots");
        for (int i = 0; i < GAMMAX_ASYNC_SLOTS; ++i) {
            if (hipEventCreateWithFlags(&sl[i].ev, hipEventDisableTiming) != hipSuccess) {
                for (int k = 0; k < i; ++k) (void)hipEventDestroy(sl[k].ev);
                delete[] sl;
                return fail(c, GAMMAX_E_DEVICE, "hipEventCreateWithFlags failed");
            }
        }
        c->slots = sl;
    }
    const int i = (int)(c->next_ticket % GAMMAX_ASYNC_SLOTS);
    AsyncSlot& sl = c->slots[i];
    if (sl.ticket)
        return fail(c, GAMMAX_E_PARAM, "GAMMAX_ASYNC_SLOTS maps are in flight: collect one with gammax_map_wait");
    hipStream_t s = (hipStream_t)stream;
    sl.p = *p;
    sl.o = opt;
    sl.ref = ref;
    sl.eval = ev;
    sl.gamma = gamma;
    sl.stream = s;
    sl.learned = learned;
    if (steady_table(c, p)) {
        // the whole map (its last kernel publishes the scalars to ring slot r); nothing waits
        CallSetup cs{p, &opt, ref, ev, gamma, n};
        const int r = claim_ring(c);
        if ((st = enqueue_steady(c, cs, false, s)) != GAMMAX_OK) return st;
        ++c->seq;
        sl.ring = r;
        HIPCHK(c, hipEventRecord(sl.ev, s));
        sl.done = false;
    } else {
        // no table for this geometry yet: the map runs to completion here (it builds one)
        if ((st = gammax_map(c, p, &opt, ref, ev, gamma, &sl.res, stream)) != GAMMAX_OK) return st;
        sl.done = true;
    }
    sl.ticket = c->next_ticket++;
    *ticket = sl.ticket;
    return GAMMAX_OK;
}

gammax_status_t gammax_map_wait(gammax_ctx_t* c, uint64_t ticket, gammax_result_t* res) {
    if (!c) return GAMMAX_E_NULL;
    if (!res) return fail(c, GAMMAX_E_NULL, "result pointer is required");
    if (!c->slots || ticket == 0 || c->slots[ticket % GAMMAX_ASYNC_SLOTS].ticket != ticket)
        return fail(c, GAMMAX_E_PARAM, "unknown ticket (never issued or already collected)");
    const int i = (int)(ticket % GAMMAX_ASYNC_SLOTS);
    AsyncSlot& sl = c->slots[i];
    sl.ticket = 0;   // collected, whatever follows
    if (sl.done) {
        *res = sl.res;
        return GAMMAX_OK;
    }
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipEventSynchronize(sl.ev));
    const Scalars h = sl.ring >= 0 ? c->h_ring[sl.ring] : sl.sc;
    gammax_status_t st = scalar_errors(c, h, sl.p.norm == GAMMAX_LOCAL);
    if (st != GAMMAX_OK) return st;
    if (h.flags & FLAG_TABLE_SHORT) {
        // the radius outgrew the cached table: the map again, synchronously, on a larger one
        return gammax_map(c, &sl.p, &sl.o, sl.ref, sl.eval, sl.gamma, res, sl.stream);
    }
    std::memset(res, 0, sizeof(*res));
    fill_result_from(c, h, res, false, 0.0f, sl.learned);
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
    if ((st = grow_work(c, n)) != GAMMAX_OK) return st;
    if ((st = grow(c, &c->hist, &c->hist_cap, sort_hist_words(n))) != GAMMAX_OK) return st;
    if (n <= SMALL_SORT_CAP) {
        // short lists: the one-workgroup rank sort (count handed over on the device)
        *c->h_count = (uint32_t)n;
        HIPCHK(c, hipMemcpyAsync(c->d_count, c->h_count, sizeof(uint32_t), hipMemcpyHostToDevice, s));
        HIPCHK(c, sort_pairs_small(keys, vals, work_array(c, W_TMP_K), work_array(c, W_TMP_V), c->d_count,
                                   &c->d_sc->sort_overflow, s));
    } else {
        HIPCHK(c, radix_sort_pairs(keys, vals, work_array(c, W_TMP_K), work_array(c, W_TMP_V), n, nullptr,
                                   c->hist, s));
    }
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

namespace {

gammax_status_t predict_nodes(gammax_ctx_t* c, gammax_model_t* m, const gammax_problem_t* p, const float* ref,
                              const float* ev, const uint32_t* nodes, int64_t n, float* y, void* stream, bool pooled) {
    if (!c) return GAMMAX_E_NULL;
    if (!m || !y || (!nodes && n > 0)) return fail(c, GAMMAX_E_NULL, "model, nodes and output are required");
    if (m->device != c->device) return fail(c, GAMMAX_E_PARAM, "model and context live on different devices");
    int o[3];
    int64_t total = 0;
    gammax_status_t st = model_inputs(c, p, ref, ev, o, &total);
    if (st != GAMMAX_OK) return st;
    if (n < 0 || n > total) return fail(c, GAMMAX_E_PARAM, "n must lie in [0, number of grid nodes]");
    if (n == 0) return GAMMAX_OK;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    if (pooled && (st = grow_pooled(c, p)) != GAMMAX_OK) return st;
    if ((st = enqueue_dose_scalars(c, p, ref, ev, total, s)) != GAMMAX_OK) return st;
    *c->h_count = (uint32_t)n;
    HIPCHK(c, hipMemcpyAsync(c->d_count, c->h_count, sizeof(uint32_t), hipMemcpyHostToDevice, s));
    TailCnnHook h{};
    h.model = m;
    h.ref = ref;
    h.ev = ev;
    for (int i = 0; i < 3; ++i) h.shape[i] = o[i];
    h.sc = c->d_sc;
    h.nodes = nodes;
    h.count = c->d_count;
    h.y = y;
    h.blocks = kTailCnnBlocks;
    if (pooled) set_pooled(c, &h);
    HIPCHK(c, tail_cnn_hook(&h, s));
    HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return device_errors(c, false);
}

}  // namespace

namespace {

gammax_status_t map_grids_2d(gammax_ctx_t* c, const gammax_problem_t* p, const gammax_grid_t* eg, const float* ref,
                             const float* ev, float* gamma, const gammax_options_t* opt, gammax_result_t* res,
                             void* stream);

}  // namespace

extern "C" {

gammax_status_t gammax_map_grids(gammax_ctx_t* c, const gammax_problem_t* p, const gammax_grid_t* eg,
                                 const float* ref, const float* ev, float* gamma, const gammax_options_t* opt_in,
                                 gammax_result_t* res, void* stream) {
    if (!c) return GAMMAX_E_NULL;
    if (!ref || !ev || !gamma || !eg) return fail(c, GAMMAX_E_NULL, "dose, gamma and grid pointers are required");
    int64_t nr = 0;
    gammax_status_t st = check_problem(c, p, &nr);
    if (st != GAMMAX_OK) return st;
    if (p->ndim == 2) return map_grids_2d(c, p, eg, ref, ev, gamma, opt_in, res, stream);
    int64_t ne = 1;
    for (int i = 0; i < 3; ++i) {
        if (eg->shape[i] < 2 || eg->shape[i] > ((int64_t)1 << 30))
            return fail(c, GAMMAX_E_SHAPE, "every evaluation axis needs at least 2 nodes");
        ne *= eg->shape[i];
        if (ne >= ((int64_t)1 << 31)) return fail(c, GAMMAX_E_SHAPE, "evaluation grid must hold < 2^31 nodes");
        if (!finite_pos(eg->spacing_mm[i])) return fail(c, GAMMAX_E_PARAM, "evaluation spacing must be finite and > 0");
        if (!std::isfinite(eg->origin_mm[i])) return fail(c, GAMMAX_E_PARAM, "evaluation origin must be finite");
    }
    if ((const float*)gamma == ref || (const float*)gamma == ev)
        return fail(c, GAMMAX_E_PARAM, "gamma must not alias the dose arrays");
    gammax_options_t opt;
    if (opt_in) opt = *opt_in;
    else gammax_options_default(&opt);
    if ((st = check_options(c, &opt)) != GAMMAX_OK) return st;
    if (opt.radius_mode != GAMMAX_RADIUS_PLAIN || opt.sort_mode != GAMMAX_SORT_NONE || opt.timing ||
        opt.tail_lanes == 1 || opt.cnn_pool || opt.projection)
        return fail(c, GAMMAX_E_PARAM, "two grids: plain radius, no sort, no timing, lanes 0 or 8..64 only");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    if ((st = grow(c, &c->g_work, &c->g_work_cap, 5 * nr)) != GAMMAX_OK) return st;
    if ((st = grow(c, &c->part, &c->part_cap, 2 * MAX_BLOCKS)) != GAMMAX_OK) return st;
    GridsArgs a{};
    a.ref = ref;
    a.ev = ev;
    a.gamma = gamma;
    for (int i = 0; i < 3; ++i) {
        a.rn[i] = (int)p->shape[i];
        a.en[i] = (int)eg->shape[i];
        a.rh[i] = p->spacing_mm[i];
        a.eh[i] = eg->spacing_mm[i];
        a.eo[i] = eg->origin_mm[i];
    }
    a.dta = p->dta_mm;
    a.dd = p->dd;
    a.thr = (float)p->dose_threshold;
    a.local = p->norm == GAMMAX_LOCAL ? 1 : 0;
    {
        // kappa(Gram) <= (s_max^2 / s_min^2) * Den in the chain basis (evaluation spacing)
        double smin = INFINITY, smax = 0.0;
        for (int i = 0; i < 3; ++i) {
            smin = std::min(smin, eg->spacing_mm[i]);
            smax = std::max(smax, eg->spacing_mm[i]);
        }
        const double guard = opt.cond_threshold * (smin * smin) / (smax * smax);
        a.den_guard = opt.precision == GAMMAX_PREC_GUARDED ? (float)guard : INFINITY;
    }
    a.sc = c->d_sc;
    a.list = c->g_work;
    a.f0 = reinterpret_cast<float*>(c->g_work + nr);
    a.guard_list = c->g_work + 2 * nr;
    a.tail_list = c->g_work + 3 * nr;
    a.tail_f = reinterpret_cast<float*>(c->g_work + 4 * nr);
    a.part = c->part;
    // the lower-key table of the evaluation grid, cached while it reaches far enough
    TableGeom g{};
    g.ndim = 3;
    g.lower = 1;
    for (int i = 0; i < 3; ++i) {
        g.shape[i] = eg->shape[i];
        g.s[i] = eg->spacing_mm[i] / p->dta_mm;
    }
    const int lanes = opt.tail_lanes > 0 ? opt.tail_lanes : 16;
    // the key-0 pass, the walk and the guard over the listed nodes (their count is on the
    // device); with no table (every first bound is 0) the key-0 pass finishes every node
    auto search = [&](const TabEntry* tab, int tab_len, float k1) -> hipError_t {
        a.tab = tab;
        a.tab_len = tab_len;
        a.k1 = k1;
        hipError_t e;
        if (opt.precision == GAMMAX_PREC_FP64) {
            if ((e = launch_grids_walk(a, opt.precision, false, lanes, s)) != hipSuccess) return e;
        } else {
            // the 27 key-0 cells one lane per node, then the walk of the nodes left
            if ((e = launch_grids_zero(a, opt.precision, s)) != hipSuccess) return e;
            if ((e = launch_grids_tail(a, opt.precision, lanes, s)) != hipSuccess) return e;
        }
        if (opt.precision == GAMMAX_PREC_GUARDED) return launch_grids_walk(a, opt.precision, true, lanes, s);
        return hipSuccess;
    };
    bool done = false;
    if (c->g_tab_valid && same_geom(c->g_geom, g)) {
        // a cached table for this geometry: the whole map on it, read back once at the end;
        // if the radius found has outgrown the table, the map runs again below on a new one
        HIPCHK(c, hipMemsetAsync(c->d_sc, 0, sizeof(Scalars), s));
        HIPCHK(c, launch_grids_prep(a, s));
        HIPCHK(c, search(c->g_tab, (int)c->g_tab_len, c->g_k1));
        HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        if ((st = scalar_errors(c, *c->h_sc, a.local != 0)) != GAMMAX_OK) return st;
        done = !((double)u2f(c->h_sc->r2_bits) >= c->g_geom.r2_cap && c->h_sc->n_masked > 0);
    }
    if (!done) {
        HIPCHK(c, hipMemsetAsync(c->d_sc, 0, sizeof(Scalars), s));
        HIPCHK(c, launch_grids_prep(a, s));
        HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        if ((st = scalar_errors(c, *c->h_sc, a.local != 0)) != GAMMAX_OK) return st;
        const float r2f = u2f(c->h_sc->r2_bits);
        if (c->h_sc->n_masked > 0 && r2f > 0.0f) {
            const bool fits = c->g_tab_valid && same_geom(c->g_geom, g) && (double)r2f < c->g_geom.r2_cap;
            if (!fits) {
                c->g_tab_valid = false;
                g.r2_cap = (double)r2f * 1.5;
                if ((st = build_rows(c, g, &c->g_tab, &c->g_tab_cap, &c->g_tab_len, &c->g_k1, s)) != GAMMAX_OK)
                    return st;
                c->g_geom = g;
                c->g_tab_valid = true;
            }
            HIPCHK(c, search(c->g_tab, (int)c->g_tab_len, c->g_k1));
        } else if (c->h_sc->n_masked > 0) {
            HIPCHK(c, search(nullptr, 0, INFINITY));
        }
        HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
    }
    const float r2 = u2f(c->h_sc->r2_bits);
    if (res) {
        const Scalars& h = *c->h_sc;
        std::memset(res, 0, sizeof(*res));
        res->n_evaluated = h.n_masked;
        res->n_pass = h.n_pass;
        res->n_borderline = h.n_border;
        res->n_cells = h.n_cells;
        res->n_guarded = h.n_guard;
        res->pass_rate = h.n_masked ? (double)h.n_pass / (double)h.n_masked : NAN;
        res->max_gamma = std::sqrt(u2f(h.maxg2_bits));
        res->dose_max = ord_to_float(h.dmax_ord);
        res->search_radius = std::sqrt(u2f(h.r2_bits));
        res->table_len = h.n_masked > 0 && r2 > 0.0f ? (int32_t)c->g_tab_len : 0;
    }
    return GAMMAX_OK;
}

}  // extern "C"

namespace {

// A 2D two-grid map as the 3D map of the pair extruded to two layers along a new slowest
// axis: the evaluation dose repeated on both layers, the reference dose on layer 0 and the
// second layer below any threshold, so only layer 0 is evaluated.  The Kuhn interpolant of a
// dose constant along that axis is the 2D interpolant at every height, so a layer-0 node's
// nearest surface point lies in its own layer and its gamma is the 2D gamma.
gammax_status_t map_grids_2d(gammax_ctx_t* c, const gammax_problem_t* p, const gammax_grid_t* eg, const float* ref,
                             const float* ev, float* gamma, const gammax_options_t* opt, gammax_result_t* res,
                             void* stream) {
    int64_t ne = 1;
    for (int i = 0; i < 2; ++i) {
        if (eg->shape[i] < 2 || eg->shape[i] > ((int64_t)1 << 30))
            return fail(c, GAMMAX_E_SHAPE, "every evaluation axis needs at least 2 nodes");
        ne *= eg->shape[i];
        if (!finite_pos(eg->spacing_mm[i])) return fail(c, GAMMAX_E_PARAM, "evaluation spacing must be finite and > 0");
        if (!std::isfinite(eg->origin_mm[i])) return fail(c, GAMMAX_E_PARAM, "evaluation origin must be finite");
    }
    const int64_t nr = p->shape[0] * p->shape[1];
    if (2 * nr >= ((int64_t)1 << 31) || 2 * ne >= ((int64_t)1 << 31))
        return fail(c, GAMMAX_E_SHAPE, "grid must hold < 2^30 nodes in 2D");
    if ((const float*)gamma == ref || (const float*)gamma == ev)
        return fail(c, GAMMAX_E_PARAM, "gamma must not alias the dose arrays");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    gammax_status_t st;
    if ((st = grow(c, &c->g_2d, &c->g_2d_cap, 4 * nr + 2 * ne)) != GAMMAX_OK) return st;
    float* ref3 = c->g_2d;
    float* gam3 = c->g_2d + 2 * nr;
    float* ev3 = c->g_2d + 4 * nr;
    const size_t rb = sizeof(float) * (size_t)nr, eb = sizeof(float) * (size_t)ne;
    HIPCHK(c, hipMemcpyAsync(ref3, ref, rb, hipMemcpyDeviceToDevice, s));
    // bytes 0x80: -1.18e-38 per node, below every threshold (and not > 0 for local
    // normalisation), and never the maximum of a pair that has a positive dose
    HIPCHK(c, hipMemsetAsync(ref3 + nr, 0x80, rb, s));
    HIPCHK(c, hipMemcpyAsync(ev3, ev, eb, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(ev3 + ne, ev, eb, hipMemcpyDeviceToDevice, s));
    const double hz = std::fmax(p->spacing_mm[0], p->spacing_mm[1]);   // any positive height
    gammax_problem_t p3 = *p;
    p3.ndim = 3;
    p3.shape[0] = 2;
    p3.shape[1] = p->shape[0];
    p3.shape[2] = p->shape[1];
    p3.spacing_mm[0] = hz;
    p3.spacing_mm[1] = p->spacing_mm[0];
    p3.spacing_mm[2] = p->spacing_mm[1];
    gammax_grid_t g3{};
    g3.shape[0] = 2;
    g3.shape[1] = eg->shape[0];
    g3.shape[2] = eg->shape[1];
    g3.spacing_mm[0] = hz;
    g3.spacing_mm[1] = eg->spacing_mm[0];
    g3.spacing_mm[2] = eg->spacing_mm[1];
    g3.origin_mm[0] = 0.0;
    g3.origin_mm[1] = eg->origin_mm[0];
    g3.origin_mm[2] = eg->origin_mm[1];
    if ((st = gammax_map_grids(c, &p3, &g3, ref3, ev3, gam3, opt, res, stream)) != GAMMAX_OK) return st;
    HIPCHK(c, hipMemcpyAsync(gamma, gam3, rb, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return GAMMAX_OK;
}

}  // namespace

extern "C" {

gammax_status_t gammax_model_features(gammax_ctx_t* c, const gammax_problem_t* p, const float* ref,
                                      const float* ev, uint16_t* feat, void* stream) {
    if (!c) return GAMMAX_E_NULL;
    if (!feat) return fail(c, GAMMAX_E_NULL, "feature buffer is required");
    int o[3];
    int64_t n = 0;
    gammax_status_t st = model_inputs(c, p, ref, ev, o, &n);
    if (st != GAMMAX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    if ((st = enqueue_dose_scalars(c, p, ref, ev, n, s)) != GAMMAX_OK) return st;
    HIPCHK(c, launch_features(ref, ev, o, c->d_sc, feat, s));
    HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return device_errors(c, false);
}

gammax_status_t gammax_model_predict(gammax_ctx_t* c, gammax_model_t* m, const gammax_problem_t* p,
                                     const float* ref, const float* ev, float* y, void* stream) {
    if (!c) return GAMMAX_E_NULL;
    if (!m || !y) return fail(c, GAMMAX_E_NULL, "model and output are required");
    if (m->device != c->device) return fail(c, GAMMAX_E_PARAM, "model and context live on different devices");
    int o[3];
    int64_t n = 0;
    gammax_status_t st = model_inputs(c, p, ref, ev, o, &n);
    if (st != GAMMAX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    CnnWs w;
    if ((st = grow_cnn(c, o, &w)) != GAMMAX_OK) return st;
    if ((st = enqueue_dose_scalars(c, p, ref, ev, n, s)) != GAMMAX_OK) return st;
    HIPCHK(c, launch_features(ref, ev, o, c->d_sc, w.feat, s));
    HIPCHK(c, model_forward(m, w.feat, 1, o, nullptr, w.a2, w.a3, y, s));
    HIPCHK(c, hipMemcpyAsync(c->h_sc, c->d_sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return device_errors(c, false);
}

gammax_status_t gammax_model_predict_nodes(gammax_ctx_t* c, gammax_model_t* m, const gammax_problem_t* p,
                                           const float* ref, const float* ev, const uint32_t* nodes, int64_t n,
                                           float* y, void* stream) {
    return predict_nodes(c, m, p, ref, ev, nodes, n, y, stream, false);
}

gammax_status_t gammax_model_predict_nodes_pooled(gammax_ctx_t* c, gammax_model_t* m, const gammax_problem_t* p,
                                                  const float* ref, const float* ev, const uint32_t* nodes, int64_t n,
                                                  float* y, void* stream) {
    return predict_nodes(c, m, p, ref, ev, nodes, n, y, stream, true);
}

}  // extern "C"

// ---- batches -----------------------------------------------------------------------------
//
// gammax_batch: the whole batch as one captured HIP graph on one stream.  Each pair keeps a
// context of its own (cell table, workspace, scalars ring).  When every pair takes the
// default pipeline (no tail sort, plain radius, FP32 or guarded precision, grouped tail
// lanes), the graph holds one launch per phase over all pairs, each block running one
// (pair, block) item of that phase's body:
//   dose maximum -> masked count -> ordered emit -> key-0 pass (items in cost order: 3D
//   pairs first, larger pairs first) -> tail walk -> FP64 guard and count reduction (each
//   pair's block 0 then stamps the device clock: completion times) -> scalars to each
//   pair's ring.
// Otherwise it holds every pair's compaction, the one key-0 launch, then every pair's own
// pipeline after the key-0 pass (network, sort, tail, guard, counts, stamp), pair by pair.
// A repeated batch replays the graph.  The tail layout of each shape class can be tuned by
// timing that layout's walk on a pair of the class (gammax_tune_*).

struct BatchState {
    std::vector<gammax_ctx*> subs;               // a context per pair index
    BatchPair* d_pairs = nullptr;                // device: pair descriptors, then the item lists
    int64_t desc_cap = 0;                        // bytes
    unsigned char* h_stage = nullptr;            // pinned: descriptors and items to upload
    int64_t stage_cap = 0;
    std::vector<unsigned char> staged_key;       // batch key of what the device holds
    unsigned long long* d_done = nullptr;        // completion clocks per pair, [n] = start
    unsigned long long* h_done = nullptr;        // pinned copy
    int64_t done_cap = 0;
    hipGraphExec_t graph = nullptr;
    std::vector<unsigned char> graph_key;
    std::map<uint64_t, int> tune;                // shape class -> lanes per node of the tail walk
    int clock_khz = 0;
};

void destroy_batch(gammax_ctx* c) {
    BatchState* b = c->batch;
    if (!b) return;
    if (b->graph) (void)hipGraphExecDestroy(b->graph);
    for (gammax_ctx* sub : b->subs) (void)gammax_ctx_destroy(sub);
    if (b->d_pairs) (void)hipFree(b->d_pairs);
    if (b->d_done) (void)hipFree(b->d_done);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    if (b->h_done) (void)hipHostFree(b->h_done);
    delete b;
    c->batch = nullptr;
}

void destroy_many(gammax_ctx* c) {
    ManyState* m = c->many;
    if (!m) return;
    for (gammax_ctx* sub : m->subs) (void)gammax_ctx_destroy(sub);
    for (auto& st : m->streams)
        if (st) (void)hipStreamDestroy(st);
    if (m->ev_in) (void)hipEventDestroy(m->ev_in);
    for (auto& e : m->ev_out)
        if (e) (void)hipEventDestroy(e);
    delete m;
    c->many = nullptr;
}

namespace {

// Shape class of a pair for the tuner: dimensionality, log2 of the node count, DD in
// 0.1 %, DTA in 0.1 mm, smallest spacing in 0.1 mm.
uint64_t shape_class(const gammax_problem_t* p, int64_t n) {
    int lg = 0;
    while (((int64_t)1 << (lg + 1)) <= n) ++lg;
    double hmin = p->spacing_mm[0];
    for (int i = 1; i < p->ndim; ++i) hmin = std::fmin(hmin, p->spacing_mm[i]);
    const uint64_t dd = (uint64_t)std::llround(p->dd * 1000.0) & 0xFFFF;
    const uint64_t dta = (uint64_t)std::llround(p->dta_mm * 10.0) & 0xFFFF;
    const uint64_t h = (uint64_t)std::llround(hmin * 10.0) & 0xFFFF;
    return (uint64_t)p->ndim | ((uint64_t)lg << 2) | (dd << 8) | (dta << 24) | (h << 40);
}

// One batch as the graph sees it: per pair its call set-up and options; the item lists of
// its launches (byte offsets and counts within the staged block after the descriptors).
struct BatchPlan {
    int n = 0;
    std::vector<gammax_options_t> opt;
    std::vector<CallSetup> cs;
    std::vector<int64_t> nodes;
    bool key0 = true;          // false for FP64 precision (its walk starts at row 0)
    bool phased = false;       // every phase one launch over all pairs (the default pipeline)
    enum { L_KEY0, L_DM, L_TILES, L_TAIL, L_FIN, kLists };
    int64_t off[kLists] = {};  // byte offset of each item list
    int count[kLists] = {};
    int64_t desc_bytes = 0;    // descriptors, then the item lists
};

int64_t descs_bytes(int n) { return (int64_t)((sizeof(BatchPair) * n + 255) / 256 * 256); }

// Whether a pair's map takes the default pipeline that the phased batch runs.
bool default_pipeline(const gammax_problem_t* p, const gammax_options_t& o) {
    return o.sort_mode == GAMMAX_SORT_NONE && !uses_model(p, &o) && o.precision != GAMMAX_PREC_FP64 &&
           o.tail_lanes != 1 && o.cell_lanes <= 1 && o.projection == 0;
}

// Lanes request of a pair's tail walk (as enqueue_search / tail_pass choose it).
int tail_g_req(const gammax_ctx* sub, const gammax_options_t& o) {
    const int tm = tail_min_lanes(sub);
    return o.tail_lanes ? o.tail_lanes : -(tm > 8 ? tm : 8);
}

// Item counts of every list and the staged size.
gammax_status_t plan_lists(gammax_ctx* c, BatchState* b, BatchPlan& P) {
    int64_t cnt[BatchPlan::kLists] = {};
    for (int i = 0; i < P.n; ++i) {
        const int64_t nn = P.nodes[i];
        cnt[BatchPlan::L_KEY0] += (nn + 255) / 256;
        if (!P.phased) continue;
        gammax_ctx* sub = b->subs[i];
        const int first = P.cs[i].p->ndim == 3 ? 8 : 4;
        cnt[BatchPlan::L_DM] += prep_reduce_blocks(nn);
        cnt[BatchPlan::L_TILES] += prep_tiles(nn);
        if (sub->tab_valid && sub->tab_len > first)
            cnt[BatchPlan::L_TAIL] += tail_grid_blocks((uint32_t)nn, tail_g_req(sub, P.opt[i]));
        const bool guarded = P.opt[i].precision == GAMMAX_PREC_GUARDED && P.cs[i].p->ndim == 3;
        cnt[BatchPlan::L_FIN] += guarded ? guard_grid_blocks() : 1;
    }
    if (!P.key0) cnt[BatchPlan::L_KEY0] = 0;
    int64_t off = descs_bytes(P.n);
    for (int k = 0; k < BatchPlan::kLists; ++k) {
        if (cnt[k] >= ((int64_t)1 << 31)) return fail(c, GAMMAX_E_SHAPE, "batch holds too many nodes");
        P.off[k] = off;
        P.count[k] = (int)cnt[k];
        off += (int64_t)sizeof(uint2) * cnt[k];
    }
    P.desc_bytes = off > descs_bytes(P.n) ? off : descs_bytes(P.n) + (int64_t)sizeof(uint2);
    return GAMMAX_OK;
}

// The descriptors of every pair (the arguments its own pipeline uses) and the item lists,
// into the pinned staging area.
void stage_batch(BatchState* b, const BatchPlan& P) {
    BatchPair* d = (BatchPair*)b->h_stage;
    std::memset(b->h_stage, 0, (size_t)P.desc_bytes);
    for (int i = 0; i < P.n; ++i) {
        gammax_ctx* c = b->subs[i];
        const gammax_problem_t* p = P.cs[i].p;
        const float r2_cap = round_down_float(c->tab_geom.r2_cap);
        d[i].sa = make_search_args(p, P.opt[i], P.cs[i].ref, P.cs[i].ev, P.cs[i].gamma, c->d_sc, c->tab,
                                   c->tab_valid ? (int)c->tab_len : 0, c->tab_valid ? c->tab_k1 : INFINITY,
                                   r2_cap, c->work, c->work_cap, c->sums, c->yhat);
        d[i].zg = make_zero_geo(p);
        d[i].pa = make_prep_args(c, P.cs[i]);
        d[i].ndim = p->ndim;
        d[i].guarded = (P.opt[i].precision == GAMMAX_PREC_GUARDED && p->ndim == 3) ? 1 : 0;
        d[i].nbr = prep_reduce_blocks(P.nodes[i]);
        d[i].first = p->ndim == 3 ? 8 : 4;
        d[i].g_req = tail_g_req(c, P.opt[i]);
        d[i].tail_blocks = (int)tail_grid_blocks((uint32_t)P.nodes[i], d[i].g_req);
        d[i].walk = (c->tab_valid && c->tab_len > d[i].first) ? 1 : 0;
        d[i].seq = c->d_seq;
        d[i].ring = c->h_ring;
        d[i].done = b->d_done + i;
    }
    // pairs in cost order for the key-0 and tail launches (3D first, larger first)
    std::vector<int> order(P.n);
    for (int i = 0; i < P.n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const double cx = (double)P.nodes[x] * (P.cs[x].p->ndim == 3 ? 8.0 : 2.0);
        const double cy = (double)P.nodes[y] * (P.cs[y].p->ndim == 3 ? 8.0 : 2.0);
        return cx > cy;
    });
    auto list = [&](int k) { return (uint2*)(b->h_stage + P.off[k]); };
    int k = 0;
    if (P.key0) {
        uint2* it = list(BatchPlan::L_KEY0);
        for (int i : order)
            for (int64_t blk = 0; blk < (P.nodes[i] + 255) / 256; ++blk) it[k++] = make_uint2((uint32_t)i, (uint32_t)blk);
    }
    if (!P.phased) return;
    uint2* dm = list(BatchPlan::L_DM);
    uint2* tiles = list(BatchPlan::L_TILES);
    uint2* tail = list(BatchPlan::L_TAIL);
    uint2* fin = list(BatchPlan::L_FIN);
    int ndm = 0, nt = 0, ntail = 0, nfin = 0;
    for (int i : order) {
        for (int j = 0; j < d[i].nbr; ++j) dm[ndm++] = make_uint2((uint32_t)i, (uint32_t)j);
        for (int64_t t = 0; t < prep_tiles(P.nodes[i]); ++t) tiles[nt++] = make_uint2((uint32_t)i, (uint32_t)t);
        if (d[i].walk)
            for (int j = 0; j < d[i].tail_blocks; ++j) tail[ntail++] = make_uint2((uint32_t)i, (uint32_t)j);
        const int nf = d[i].guarded ? (int)guard_grid_blocks() : 1;
        for (int j = 0; j < nf; ++j) fin[nfin++] = make_uint2((uint32_t)i, (uint32_t)j);
    }
}

// Queue the whole batch on `s` (the capture stream, or the caller's stream for a direct run).
gammax_status_t enqueue_batch(gammax_ctx* c, BatchState* b, const BatchPlan& P, hipStream_t s) {
    gammax_status_t st;
    const unsigned char* dev = (const unsigned char*)b->d_pairs;
    auto list = [&](int k) { return (const uint2*)(dev + P.off[k]); };
    HIPCHK(c, launch_stamp(b->d_done + P.n, s));
    if (P.phased) {
        HIPCHK(c, launch_batch_prep(b->d_pairs, list(BatchPlan::L_DM), P.count[BatchPlan::L_DM],
                                    list(BatchPlan::L_TILES), P.count[BatchPlan::L_TILES], s));
        HIPCHK(c, launch_batch_key0(b->d_pairs, list(BatchPlan::L_KEY0), P.count[BatchPlan::L_KEY0], s));
        HIPCHK(c, launch_batch_tail(b->d_pairs, list(BatchPlan::L_TAIL), P.count[BatchPlan::L_TAIL], s));
        HIPCHK(c, launch_batch_finish(b->d_pairs, list(BatchPlan::L_FIN), P.count[BatchPlan::L_FIN], s));
        hipLaunchKernelGGL(k_batch_publish, dim3((unsigned)P.n), dim3(64), 0, s, (const BatchPair*)b->d_pairs);
        HIPCHK(c, hipGetLastError());
        return GAMMAX_OK;
    }
    for (int i = 0; i < P.n; ++i)
        if ((st = enqueue_prep(b->subs[i], P.cs[i], s, nullptr, nullptr)) != GAMMAX_OK)
            return fail(c, st, "pair " + std::to_string(i) + ": " + b->subs[i]->err);
    if (P.key0)
        HIPCHK(c, launch_batch_key0(b->d_pairs, list(BatchPlan::L_KEY0), P.count[BatchPlan::L_KEY0], s));
    for (int i = 0; i < P.n; ++i) {
        gammax_ctx* sub = b->subs[i];
        const float r2_cap = round_down_float(sub->tab_geom.r2_cap);
        if ((st = enqueue_search(sub, P.cs[i], (uint32_t)P.nodes[i], r2_cap, s, false, P.key0)) != GAMMAX_OK)
            return fail(c, st, "pair " + std::to_string(i) + ": " + sub->err);
        HIPCHK(c, launch_stamp(b->d_done + i, s));
    }
    return GAMMAX_OK;
}

// The batch key: every pair's own graph key (pointers, problem, options and the context
// state its pipeline depends on: the descriptors and item lists derive from these), the
// plan's shape and the batch's own buffers.  Equal keys mean equal staged bytes.
std::vector<unsigned char> batch_key(BatchState* b, const BatchPlan& P) {
    std::vector<unsigned char> k;
    auto put = [&](const void* q, size_t n) {
        const unsigned char* u = (const unsigned char*)q;
        k.insert(k.end(), u, u + n);
    };
    for (int i = 0; i < P.n; ++i) {
        const GraphKey g = key_of(b->subs[i], P.cs[i]);
        put(&g, sizeof(g));
    }
    const void* bufs[2] = {b->d_pairs, b->d_done};
    put(bufs, sizeof(bufs));
    const int flags[2] = {P.key0 ? 1 : 0, P.phased ? 1 : 0};
    put(flags, sizeof(flags));
    put(P.count, sizeof(P.count));
    return k;
}

// Run the batch once (replaying the graph when possible), ring slots claimed and counted
// as every pair's map publishes its scalars.  ring[i] receives pair i's slot.  The
// descriptors and item lists are staged and uploaded only when the batch key changes.
gammax_status_t launch_batch(gammax_ctx* c, BatchState* b, const BatchPlan& P, hipStream_t s,
                             std::vector<int>& ring) {
    gammax_status_t st;
    const std::vector<unsigned char> key = batch_key(b, P);
    if (key != b->staged_key) {
        stage_batch(b, P);
        HIPCHK(c, hipMemcpyAsync(b->d_pairs, b->h_stage, (size_t)P.desc_bytes, hipMemcpyHostToDevice, s));
        b->staged_key = key;
    }
    for (int i = 0; i < P.n; ++i) ring[i] = claim_ring(b->subs[i]);
    bool launched = false;
    if (!c->graph_broken) {
        if (!b->graph || key != b->graph_key) {
            if (b->graph) (void)hipGraphExecDestroy(b->graph);
            b->graph = nullptr;
            if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
            HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            st = enqueue_batch(c, b, P, c->cap_stream);
            hipGraph_t g = nullptr;
            const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
            if (st == GAMMAX_OK && e == hipSuccess && g && hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0) == hipSuccess) {
                b->graph_key = key;
            } else {
                b->graph = nullptr;
                c->graph_broken = true;   // launch directly from now on
                (void)hipGetLastError();
            }
            if (g) (void)hipGraphDestroy(g);
            if (st != GAMMAX_OK) return st;
        }
        if (b->graph) {
            HIPCHK(c, hipGraphLaunch(b->graph, s));
            launched = true;
        }
    }
    if (!launched && (st = enqueue_batch(c, b, P, s)) != GAMMAX_OK) return st;
    for (int i = 0; i < P.n; ++i) ++b->subs[i]->seq;
    return GAMMAX_OK;
}

}  // namespace

namespace {

// The maps of n pairs queued on the caller's stream and three internal ones (a cached
// context per pair index), then collected.
gammax_status_t run_many(gammax_ctx_t* c, int32_t n, const gammax_problem_t* probs, const float* const* refs,
                         const float* const* evals, float* const* gammas, const gammax_options_t* opt,
                         gammax_result_t* results, hipStream_t s) {
    if (!c) return GAMMAX_E_NULL;
    if (n < 0) return fail(c, GAMMAX_E_PARAM, "n must be >= 0");
    if (n == 0) return GAMMAX_OK;
    if (!probs || !refs || !evals || !gammas || !results)
        return fail(c, GAMMAX_E_NULL, "problems, dose, gamma and result arrays are required");
    if (opt && opt->timing) return fail(c, GAMMAX_E_PARAM, "timing is not available for gammax_map_many");
    if (opt && opt->sort_mode == GAMMAX_SORT_GIVEN)
        return fail(c, GAMMAX_E_PARAM, "the given order is for single maps (one key array per grid)");
    HIPCHK(c, hipSetDevice(c->device));
    if (!c->many) {
        ManyState* m = new (std::nothrow) ManyState();
        if (!m) return fail(c, GAMMAX_E_NOMEM, "gammax_map_many state");
        c->many = m;
        for (auto& st : m->streams) HIPCHK(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&m->ev_in, hipEventDisableTiming));
        for (auto& e : m->ev_out) HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    ManyState* m = c->many;
    while ((int)m->subs.size() < n) {
        gammax_ctx* sub = nullptr;
        const gammax_status_t st = gammax_ctx_create(c->device, &sub);
        if (st != GAMMAX_OK) return fail(c, st, "gammax_map_many: context for a pair");
        m->subs.push_back(sub);
    }
    // the internal streams start after the caller's work on `stream`
    HIPCHK(c, hipEventRecord(m->ev_in, s));
    for (auto& st : m->streams) HIPCHK(c, hipStreamWaitEvent(st, m->ev_in, 0));
    std::vector<uint64_t> tickets(n, 0);
    gammax_status_t first = GAMMAX_OK;
    std::string why;
    int queued = 0;
    for (int i = 0; i < n; ++i) {
        const int k = i % kManyStreams;
        hipStream_t si = k == 0 ? s : m->streams[k - 1];
        const gammax_status_t st = gammax_map_async(m->subs[i], &probs[i], opt, refs[i], evals[i], gammas[i],
                                                    &tickets[i], si);
        if (st != GAMMAX_OK) {
            first = st;
            why = "pair " + std::to_string(i) + ": " + m->subs[i]->err;
            break;
        }
        ++queued;
    }
    for (int i = 0; i < queued; ++i) {
        const gammax_status_t st = gammax_map_wait(m->subs[i], tickets[i], &results[i]);
        if (st != GAMMAX_OK && first == GAMMAX_OK) {
            first = st;
            why = "pair " + std::to_string(i) + ": " + m->subs[i]->err;
        }
    }
    // later work on the caller's stream follows the maps
    for (int k = 0; k < kManyStreams - 1; ++k) {
        HIPCHK(c, hipEventRecord(m->ev_out[k], m->streams[k]));
        HIPCHK(c, hipStreamWaitEvent(s, m->ev_out[k], 0));
    }
    if (first != GAMMAX_OK) return fail(c, first, why);
    return GAMMAX_OK;
}

}  // namespace

extern "C" {

gammax_status_t gammax_batch(gammax_ctx_t* c, int32_t n, const gammax_problem_t* probs, const float* const* refs,
                             const float* const* evals, float* const* gammas, const gammax_options_t* opt_in,
                             gammax_result_t* results, void* stream) {
    if (!c) return GAMMAX_E_NULL;
    if (n < 0) return fail(c, GAMMAX_E_PARAM, "n must be >= 0");
    if (n == 0) return GAMMAX_OK;
    if (!probs || !refs || !evals || !gammas || !results)
        return fail(c, GAMMAX_E_NULL, "problems, dose, gamma and result arrays are required");
    gammax_options_t opt;
    if (opt_in) opt = *opt_in;
    else gammax_options_default(&opt);
    gammax_status_t st = check_options(c, &opt);
    if (st != GAMMAX_OK) return st;
    if (opt.timing) return fail(c, GAMMAX_E_PARAM, "timing is not available for gammax_batch");
    if (opt.sort_mode == GAMMAX_SORT_GIVEN)
        return fail(c, GAMMAX_E_PARAM, "the given order is for single maps (one key array per grid)");
    if (opt.projection != 0 || opt.cell_lanes > 1)
        return fail(c, GAMMAX_E_PARAM, "the batch runs the default key-0 pass (projection 0, one lane per node)");
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(c, hipSetDevice(c->device));
    if (!c->batch) {
        c->batch = new (std::nothrow) BatchState();
        if (!c->batch) return fail(c, GAMMAX_E_NOMEM, "batch state");
    }
    BatchState* b = c->batch;
    if (b->clock_khz == 0)
        HIPCHK(c, hipDeviceGetAttribute(&b->clock_khz, hipDeviceAttributeWallClockRate, c->device));
    while ((int)b->subs.size() < n) {
        gammax_ctx* sub = nullptr;
        if ((st = gammax_ctx_create(c->device, &sub)) != GAMMAX_OK) return fail(c, st, "batch: context for a pair");
        b->subs.push_back(sub);
    }

    // every pair: checks, workspace, and a cell table for its geometry (a pair met for the
    // first time runs its map once on its own context, which builds the table)
    BatchPlan P;
    P.n = n;
    P.opt.resize(n);
    P.cs.resize(n);
    P.nodes.resize(n);
    P.key0 = opt.precision != GAMMAX_PREC_FP64;
    std::vector<uint64_t> cls(n);
    std::vector<int> learned(n, 0);
    for (int i = 0; i < n; ++i) {
        gammax_ctx* sub = b->subs[i];
        int64_t nn = 0;
        if ((st = check_problem(c, &probs[i], &nn)) != GAMMAX_OK) return fail(c, st, "pair " + std::to_string(i) + ": " + c->err);
        cls[i] = shape_class(&probs[i], nn);
        gammax_options_t oi = opt;
        if (opt.tail_lanes == 0 && b->tune.count(cls[i])) oi.tail_lanes = b->tune[cls[i]];
        bool lr = false;
        if ((st = map_setup(sub, &probs[i], &oi, refs[i], evals[i], gammas[i], &P.opt[i], &nn, &lr)) != GAMMAX_OK)
            return fail(c, st, "pair " + std::to_string(i) + ": " + sub->err);
        learned[i] = lr ? 1 : 0;
        P.nodes[i] = nn;
        P.cs[i] = CallSetup{&probs[i], &P.opt[i], refs[i], evals[i], gammas[i], nn};
        if (!steady_table(sub, &probs[i])) {
            gammax_result_t r{};
            if ((st = gammax_map(sub, &probs[i], &P.opt[i], refs[i], evals[i], gammas[i], &r, s)) != GAMMAX_OK)
                return fail(c, st, "pair " + std::to_string(i) + ": " + sub->err);
            if (!sub->tab_valid) {
                // no walk needed yet (every gamma0 0, or nothing evaluated): an empty table
                // for the geometry, so that the pair takes part in the graph
                sub->tab_geom = geom_of(&probs[i]);
                sub->tab_geom.r2_cap = 0.0;
                sub->tab_len = 0;
                sub->tab_k1 = INFINITY;
                sub->tab_valid = true;
            }
        }
    }
    // tail layout of shape classes met for the first time: on the first pair of the class,
    // its own map timed with each layout (direct launches with phase events), the layout
    // whose tail walk was fastest kept
    if (opt.autotune && opt.tail_lanes == 0) {
        for (int i = 0; i < n; ++i) {
            if (b->tune.count(cls[i])) continue;
            float best_ms = INFINITY;
            int best_g = 0;
            for (int g : {0, 8, 16, 32, 64}) {
                gammax_options_t ot = P.opt[i];
                ot.tail_lanes = g;
                ot.timing = 1;
                float ms = INFINITY;
                for (int rep = 0; rep < 2; ++rep) {
                    gammax_result_t r{};
                    if ((st = gammax_map(b->subs[i], &probs[i], &ot, refs[i], evals[i], gammas[i], &r, s)) !=
                        GAMMAX_OK)
                        return fail(c, st, "pair " + std::to_string(i) + ": " + b->subs[i]->err);
                    ms = std::fmin(ms, r.ms_tail);
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best_g = g;
                }
            }
            b->tune[cls[i]] = best_g;
        }
        for (int i = 0; i < n; ++i) P.opt[i].tail_lanes = b->tune[cls[i]];
    }


    // the launches: one per phase over all pairs when every pair takes the default pipeline
    P.phased = P.key0;
    for (int i = 0; i < n; ++i) P.phased = P.phased && default_pipeline(&probs[i], P.opt[i]);
    if ((st = plan_lists(c, b, P)) != GAMMAX_OK) return st;
    if (P.desc_bytes > b->desc_cap || !b->d_pairs) {
        if (b->graph) (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
        int64_t cap = b->desc_cap;
        unsigned char* raw = (unsigned char*)b->d_pairs;
        if ((st = grow(c, &raw, &cap, P.desc_bytes)) != GAMMAX_OK) return st;
        b->d_pairs = (BatchPair*)raw;
        b->desc_cap = cap;
        b->staged_key.clear();
    }
    if (P.desc_bytes > b->stage_cap || !b->h_stage) {
        if (b->h_stage) (void)hipHostFree(b->h_stage);
        b->h_stage = nullptr;
        b->stage_cap = 0;
        HIPCHK(c, hipHostMalloc((void**)&b->h_stage, (size_t)P.desc_bytes, hipHostMallocDefault));
        b->stage_cap = P.desc_bytes;
    }
    if (n + 1 > b->done_cap || !b->d_done) {
        if (b->graph) (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
        if (b->h_done) (void)hipHostFree(b->h_done);
        b->h_done = nullptr;
        int64_t cap = b->done_cap;
        if ((st = grow(c, &b->d_done, &cap, n + 1)) != GAMMAX_OK) return st;
        b->done_cap = cap;
        HIPCHK(c, hipHostMalloc((void**)&b->h_done, sizeof(unsigned long long) * (size_t)cap, hipHostMallocDefault));
    }
    std::vector<int> ring(n, 0);

    // the batch
    if ((st = launch_batch(c, b, P, s, ring)) != GAMMAX_OK) return st;
    HIPCHK(c, hipMemcpyAsync(b->h_done, b->d_done, sizeof(unsigned long long) * (size_t)(n + 1),
                             hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const unsigned long long t0 = b->h_done[n];
    for (int i = 0; i < n; ++i) {
        gammax_ctx* sub = b->subs[i];
        const Scalars h = sub->h_ring[ring[i]];
        if ((st = scalar_errors(sub, h, probs[i].norm == GAMMAX_LOCAL)) != GAMMAX_OK)
            return fail(c, st, "pair " + std::to_string(i) + ": " + sub->err);
        gammax_result_t& r = results[i];
        std::memset(&r, 0, sizeof(r));
        if (h.flags & FLAG_TABLE_SHORT) {
            // the radius outgrew the pair's table: its map again on its own context (which
            // builds a larger table; the next batch recaptures)
            if ((st = gammax_map(sub, &probs[i], &P.opt[i], refs[i], evals[i], gammas[i], &r, s)) != GAMMAX_OK)
                return fail(c, st, "pair " + std::to_string(i) + ": " + sub->err);
        } else {
            fill_result_from(sub, h, &r, false, 0.0f, learned[i] != 0);
        }
        const unsigned long long t = b->h_done[i];
        r.ms_done = (t > t0 && b->clock_khz > 0) ? (float)((double)(t - t0) / b->clock_khz) : 0.0f;
    }
    return GAMMAX_OK;
}

gammax_status_t gammax_map_many(gammax_ctx_t* c, int32_t n, const gammax_problem_t* probs, const float* const* refs,
                                const float* const* evals, float* const* gammas, const gammax_options_t* opt,
                                gammax_result_t* results, void* stream) {
    return run_many(c, n, probs, refs, evals, gammas, opt, results, (hipStream_t)stream);
}

gammax_status_t gammax_tune_save(const gammax_ctx_t* c, const char* path) {
    if (!c || !path) return GAMMAX_E_NULL;
    FILE* f = std::fopen(path, "w");
    if (!f) return GAMMAX_E_PARAM;
    if (c->batch)
        for (const auto& kv : c->batch->tune) std::fprintf(f, "%llu %d\n", (unsigned long long)kv.first, kv.second);
    std::fclose(f);
    return GAMMAX_OK;
}

gammax_status_t gammax_tune_load(gammax_ctx_t* c, const char* path) {
    if (!c || !path) return GAMMAX_E_NULL;
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(c, GAMMAX_E_PARAM, std::string("cannot open ") + path);
    if (!c->batch) {
        c->batch = new (std::nothrow) BatchState();
        if (!c->batch) {
            std::fclose(f);
            return GAMMAX_E_NOMEM;
        }
    }
    unsigned long long k = 0;
    int g = 0;
    gammax_status_t st = GAMMAX_OK;
    while (std::fscanf(f, "%llu %d", &k, &g) == 2) {
        if (!(g == 0 || g == 1 || g == 8 || g == 16 || g == 32 || g == 64)) {
            st = fail(c, GAMMAX_E_PARAM, "bad lanes value in tuning file");
            break;
        }
        c->batch->tune[(uint64_t)k] = g;
    }
    std::fclose(f);
    return st;
}

}  // extern "C"

// ---- gammax_map_noalloc: the map without device allocations ------------------------------
//
// Every buffer the map needs beyond the caller's doses and gamma lives in `scratch`, one
// file-scope device array that each GPU holds a copy of, at an address of its own.  In host
// code the array's name is a host-side stand-in, not a device address: it is never passed to
// a kernel or a copy.  The device address is taken once per device, with that device
// current, by hipGetSymbolAddress and kept in na_ptr[device]; every launch and copy below
// uses that address.  Pieces (256-byte aligned): scalars, dose-max partials, prep tile
// counts, search partial sums, sort histogram, the table build count, the node work arrays
// (kWorkArrays x GAMMAX_NOALLOC_MAX_NODES words), the table build arrays (4 x box words) and
// the table rows.  The kernels clear what must start at zero (the prep clears the counters
// and partial sums, a one-word kernel the table count), so the contents a previous call
// left do not matter.

namespace {

constexpr int64_t kNaNodes = GAMMAX_NOALLOC_MAX_NODES;
constexpr int64_t kNaRows = GAMMAX_NOALLOC_MAX_TABLE;
constexpr int64_t kNaBox = 2 * GAMMAX_NOALLOC_MAX_TABLE;   // candidate box of the table build
constexpr int64_t kNaBytes = GAMMAX_NOALLOC_SCRATCH_BYTES;
constexpr int kNaDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNaBytes];

std::mutex na_mutex;
unsigned char* na_ptr[kNaDevices] = {};

struct NaLayout {
    Scalars* sc;
    uint32_t* part;
    uint32_t* blockcnt;
    BlockSums* sums;
    uint32_t* hist;
    uint32_t* count;
    uint32_t* work;
    uint32_t* tb;
    TabEntry* tab;
    int64_t bytes;
};

NaLayout na_layout(unsigned char* base) {
    NaLayout L{};
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        unsigned char* p = base ? base + off : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    L.sc = (Scalars*)take(sizeof(Scalars));
    L.part = (uint32_t*)take(4 * 2 * (int64_t)MAX_BLOCKS);
    L.blockcnt = (uint32_t*)take(4 * prep_words(kNaNodes));
    L.sums = (BlockSums*)take((int64_t)sizeof(BlockSums) * search_sums_needed((uint32_t)kNaNodes));
    L.hist = (uint32_t*)take(4 * sort_hist_words(kNaNodes > kNaBox ? kNaNodes : kNaBox));
    L.count = (uint32_t*)take(4);
    L.work = (uint32_t*)take(4 * (int64_t)kWorkArrays * kNaNodes);
    L.tb = (uint32_t*)take(4 * 4 * kNaBox);
    L.tab = (TabEntry*)take((int64_t)sizeof(TabEntry) * kNaRows);
    L.bytes = off;
    return L;
}

// The scratch array's address on device `dev` (the current device), taken on the first call.
gammax_status_t na_base(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kNaDevices) return GAMMAX_E_DEVICE;
    std::lock_guard<std::mutex> lock(na_mutex);
    if (!na_ptr[dev]) {
        if (na_layout(nullptr).bytes > kNaBytes) return GAMMAX_E_NOMEM;   // layout and array size disagree
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return GAMMAX_E_DEVICE;
        }
        na_ptr[dev] = (unsigned char*)p;
    }
    *out = na_ptr[dev];
    return GAMMAX_OK;
}

gammax_status_t na_read_scalars(const NaLayout& L, Scalars* h, hipStream_t s) {
    HIPCHK(nullptr, hipMemcpyAsync(h, L.sc, sizeof(Scalars), hipMemcpyDeviceToHost, s));
    HIPCHK(nullptr, hipStreamSynchronize(s));
    return GAMMAX_OK;
}

}  // namespace

extern "C" {

gammax_status_t gammax_map_noalloc(const gammax_problem_t* p, const gammax_options_t* opt_in, const float* ref,
                                   const float* ev, float* gamma, gammax_result_t* res, void* stream) {
    if (!res || !ref || !ev || !gamma) return GAMMAX_E_NULL;
    int64_t n = 0;
    gammax_status_t st = check_problem(nullptr, p, &n);
    if (st != GAMMAX_OK) return st;
    if (n > kNaNodes) return GAMMAX_E_SHAPE;
    if (gamma == ref || gamma == ev) return GAMMAX_E_PARAM;
    gammax_options_t opt;
    if (opt_in) opt = *opt_in;
    else gammax_options_default(&opt);
    if ((st = check_options(nullptr, &opt)) != GAMMAX_OK) return st;
    if (opt.timing || opt.model || opt.radius_mode != GAMMAX_RADIUS_PLAIN || opt.sort_mode == GAMMAX_SORT_PREDICTED ||
        opt.sort_mode == GAMMAX_SORT_GIVEN || opt.autotune || opt.cnn_pool)
        return GAMMAX_E_PARAM;
    int dev = 0;
    HIPCHK(nullptr, hipGetDevice(&dev));
    unsigned char* base = nullptr;
    if ((st = na_base(dev, &base)) != GAMMAX_OK) return st;
    const NaLayout L = na_layout(base);
    hipStream_t s = (hipStream_t)stream;
    std::memset(res, 0, sizeof(*res));
    const int64_t ntiles = prep_tiles(n);
    uint32_t* nodes_arr = L.work + (int64_t)W_NODES * kNaNodes;

    // compaction (Kernel 1): dose maximum, mask, gamma0, masked nodes in grid order
    PrepArgs pa{};
    pa.ref = ref;
    pa.ev = ev;
    pa.gamma = gamma;
    pa.n = n;
    pa.thr = (float)p->dose_threshold;
    pa.dd = (float)p->dd;
    pa.local = p->norm == GAMMAX_LOCAL ? 1 : 0;
    pa.sc = L.sc;
    pa.part = L.part;
    pa.blockcnt = L.blockcnt;
    prep_groups(n, &pa.super_shift, &pa.n_super);
    pa.super = L.blockcnt + ntiles;
    pa.ntiles = (int)ntiles;
    pa.nodes = nodes_arr;
    pa.sums = L.sums;
    pa.mbits = reinterpret_cast<unsigned long long*>(L.blockcnt + prep_mbits_offset(n));
    HIPCHK(nullptr, launch_prep(pa, s));
    Scalars h{};
    if ((st = na_read_scalars(L, &h, s)) != GAMMAX_OK) return st;
    if ((st = scalar_errors(nullptr, h, p->norm == GAMMAX_LOCAL)) != GAMMAX_OK) return st;
    const uint32_t M = h.n_masked;
    const float r2 = u2f(h.r2_bits);

    // the cell table for this radius (Algorithm A1 steps 2-3), built in the scratch array
    int64_t T = 0;
    float k1 = INFINITY;
    if (M > 0 && r2 > 0.0f) {
        TableGeom g = geom_of(p);
        g.r2_cap = (double)r2;   // every cell whose key is below the largest gamma0
        table_box(g);
        if (g.box > kNaBox) return GAMMAX_E_RADIUS;
        uint32_t* keys = L.tb;
        uint32_t* vals = L.tb + kNaBox;
        uint32_t* tk = L.tb + 2 * kNaBox;
        uint32_t* tv = L.tb + 3 * kNaBox;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, L.count);
        HIPCHK(nullptr, hipGetLastError());
        HIPCHK(nullptr, launch_table_gen(g, keys, vals, L.count, s));
        HIPCHK(nullptr, radix_sort_pairs(keys, vals, tk, tv, g.box, nullptr, L.hist, s));
        uint32_t rows = 0;
        HIPCHK(nullptr, hipMemcpyAsync(&rows, L.count, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(nullptr, hipStreamSynchronize(s));
        if ((int64_t)rows > kNaRows) return GAMMAX_E_RADIUS;
        HIPCHK(nullptr, launch_table_rows(g, vals, rows, L.tab, s));
        const int zero_rows = p->ndim == 3 ? 8 : 4;
        if ((int)rows > zero_rows) {
            HIPCHK(nullptr, hipMemcpyAsync(&k1, &L.tab[zero_rows].key2, sizeof(float), hipMemcpyDeviceToHost, s));
            HIPCHK(nullptr, hipStreamSynchronize(s));
        }
        T = rows;
    }

    // the search (steps 3, 6, 7) and the counts
    if (M > 0) {
        const SearchArgs sa = make_search_args(p, opt, ref, ev, gamma, L.sc, L.tab, (int)T, k1, INFINITY, L.work,
                                               kNaNodes, L.sums, nullptr);
        SearchPlan plan{};
        plan.ndim = p->ndim;
        plan.precision = opt.precision;
        plan.tail_lanes = opt.tail_lanes;
        plan.tail_min_lanes = 0;
        plan.zero_lanes = (opt.cell_lanes == 4 || opt.cell_lanes == 8) ? 1 : 0;
        plan.projection = opt.projection;
        plan.M = M;
        plan.zero = make_zero_geo(p);
        plan.tmp_keys = L.work + (int64_t)W_TMP_K * kNaNodes;
        plan.tmp_vals = L.work + (int64_t)W_TMP_V * kNaNodes;
        plan.hist = opt.sort_mode == GAMMAX_SORT_NONE ? nullptr : L.hist;
        plan.small_sort = 0;
        HIPCHK(nullptr, launch_search(sa, plan, s));
        if ((st = na_read_scalars(L, &h, s)) != GAMMAX_OK) return st;
    }
    res->n_evaluated = h.n_masked;
    res->n_pass = h.n_pass;
    res->n_borderline = h.n_border;
    res->n_fp64_tets = h.n_fp64;
    res->n_cells = h.n_cells;
    res->n_tail = h.n_tail;
    res->n_guarded = h.n_guard;
    res->pass_rate = h.n_masked ? (double)h.n_pass / (double)h.n_masked : NAN;
    res->max_gamma = std::sqrt(u2f(h.maxg2_bits));
    res->dose_max = ord_to_float(h.dmax_ord);
    res->search_radius = std::sqrt(r2);
    res->table_len = (int32_t)T;
    res->long_walk_rows = h.long_rows;
    return GAMMAX_OK;
}

}  // extern "C"
