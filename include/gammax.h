/*
 * gammax — gamma-index dose comparison on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the library libgammax.so.  Plain pointers and sizes only; no C++ exception
 * crosses it; every call returns a gammax_status_t and never aborts the process.
 *
 * Method: Gu, Jia & Jiang, "GPU-based fast gamma index calculation" (arXiv:1012.1900).
 *   gamma(r) = min over the evaluation surface of |r~ - x~|              (Sec. 2.1, Eq. (1))
 *   with r~ = (r / DTA, D_r(r) / dD); the evaluation surface is the piecewise-linear
 *   interpolant of D_e over the Kuhn triangulation of the grid (the geometric method the
 *   paper adopts), searched over a radially sorted cell table with an early break
 *   (Algorithm A1) by one lane per reference node over dose-difference-sorted nodes
 *   (Sec. 2.2, Algorithm A2).
 *
 * Grids.  Reference and evaluation doses share one regular grid.  Arrays are C-ordered
 * float32 with the fastest axis last: 3D shape = (nz, ny, nx), 2D shape = (ny, nx).
 * Node i of an axis sits at i * spacing.  Every axis needs at least 2 nodes.
 *
 * Memory.  Dose and gamma buffers are device memory owned by the caller.  The context
 * owns every scratch buffer it needs; it grows them on demand and frees them on destroy.
 * A context serves one caller at a time (not thread-safe); use one per host thread.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the default stream).  Calls that return
 * results on the host synchronise that stream before they return.
 *
 * Errors.  Argument errors are detected on the host before any launch.  Conditions that
 * only the device can see (non-finite doses, no positive reference dose) are reported
 * after the device pass that finds them; the gamma buffer is then unspecified.
 */
#ifndef GAMMAX_H
#define GAMMAX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GAMMAX_OK = 0,
    GAMMAX_E_NULL = -1,       /* a required pointer is NULL */
    GAMMAX_E_SHAPE = -2,      /* ndim not 2 or 3, an axis with < 2 nodes, or > 2^31 nodes */
    GAMMAX_E_PARAM = -3,      /* spacing, DD or DTA <= 0 (or not finite), threshold outside [0,1), bad option */
    GAMMAX_E_NONFINITE = -4,  /* a dose value is NaN or infinite */
    GAMMAX_E_NOMEM = -5,      /* device or pinned host allocation failed */
    GAMMAX_E_DEVICE = -6,     /* a HIP runtime call failed; see gammax_last_error() */
    GAMMAX_E_RADIUS = -7,     /* the cell table for this search radius exceeds the table cap */
    GAMMAX_E_DOSE = -8,       /* global normalisation with no positive reference dose */
    GAMMAX_E_MODEL = -9       /* a model file that cannot be read or written, or is not a
                                 model of this network (gammax_model_save / _load) */
} gammax_status_t;

typedef enum { GAMMAX_GLOBAL = 0, GAMMAX_LOCAL = 1 } gammax_norm_t;

/*
 * Work order of the search (Sec. 2.2; results never depend on it).  Every masked node
 * first evaluates the 2^d cells with key 0 around it, in grid order; nodes whose bound
 * then still exceeds the next key continue the walk, in this order:
 */
typedef enum {
    GAMMAX_SORT_NONE = 0,     /* as they were queued (default) */
    GAMMAX_SORT_DD = 1,       /* ascending |DD| / dD ("DD sorting", Algorithm A2 step 3) */
    GAMMAX_SORT_BOUND = 2,    /* ascending gamma bound after the key-0 cells */
    GAMMAX_SORT_PREDICTED = 3, /* ascending predicted gamma (needs a model; 3D) */
    GAMMAX_SORT_GIVEN = 4     /* ascending key given by the caller per node (options.order_key;
                                 plain radius, single maps): e.g. a known gamma, to measure
                                 what a perfect predictor's order buys */
} gammax_sort_t;

/* Search radius of the walk past the key-0 cells. */
typedef enum {
    GAMMAX_RADIUS_PLAIN = 0,  /* walk until the next key reaches the current gamma (default) */
    GAMMAX_RADIUS_LEARNED = 1 /* first walk only while the key is below radius_factor * gamma_hat
                                 (gamma_hat from the model); a node whose gamma is not certified
                                 inside that radius then finishes with the plain walk from where
                                 the first one stopped.  Results equal the plain search.  3D only;
                                 2D problems use the plain radius. */
} gammax_radius_t;

typedef struct gammax_model gammax_model_t;

/* Arithmetic of the per-simplex projections. */
typedef enum {
    GAMMAX_PREC_FP32 = 0,        /* FP32 everywhere */
    GAMMAX_PREC_GUARDED = 1,     /* FP32; a tetrahedron whose Gram matrix condition number may
                                    exceed cond_threshold is re-projected in FP64 (default) */
    GAMMAX_PREC_FP64 = 2         /* FP64 for every face */
} gammax_precision_t;

/* The problem: the paper's statement gamma_map(ref, eval, spacing, DD, DTA, threshold, norm). */
typedef struct {
    int32_t ndim;             /* 2 or 3 */
    int32_t norm;             /* gammax_norm_t: dD = DD * max(D_r) (global) or DD * D_r(r) (local) */
    int64_t shape[3];         /* slowest axis first; 2D uses shape[0..1] = (ny, nx) */
    double spacing_mm[3];     /* same axis order as shape; > 0 */
    double dd;                /* dose criterion as a fraction, e.g. 0.03 */
    double dta_mm;            /* distance-to-agreement criterion in mm, e.g. 3.0 */
    double dose_threshold;    /* low-dose cutoff as a fraction of max(D_r), in [0, 1), e.g. 0.10.
                                 Reference nodes with D_r < fl32(threshold * max D_r) are not
                                 evaluated (local normalisation also skips D_r <= 0). */
} gammax_problem_t;

typedef struct {
    int32_t sort_mode;        /* gammax_sort_t */
    int32_t precision;        /* gammax_precision_t */
    double cond_threshold;    /* condition-number bound of the FP64 guard, default 1e6 */
    int32_t timing;           /* 1: time the phases with HIP events (fills ms_* in the result) */
    int32_t tail_lanes;       /* lanes that share one node in the walk past the key-0 cells:
                                 0 = automatic, 1 = one lane per node (the paper's layout),
                                 8, 16, 32 or 64 = that many table rows of a node at once */
    int32_t cell_lanes;       /* layout of the pass over the key-0 cells: 0 = automatic
                                 (one lane per node), 1 = one lane per node, 4 (2D) or
                                 8 (3D) = one lane per cell */
    int32_t radius_mode;      /* gammax_radius_t */
    const gammax_model_t *model;  /* the model for GAMMAX_RADIUS_LEARNED / GAMMAX_SORT_PREDICTED */
    double radius_factor;     /* f of the learned radius f * gamma_hat, >= 1 (default 1.1) */
    int32_t autotune;         /* gammax_batch: 1 = time the tail layouts of each new shape class on
                                 the first call and keep the fastest (see gammax_batch) */
    int32_t cnn_pool;         /* resolution of the network input (learned radius / predicted order):
                                 0 = the grid's own (each tail node's 9^3 patch);
                                 2 = the pair average-pooled 2x2x2 (a grid at half the model's
                                 training spacing), the network over the whole coarse grid and
                                 gamma_hat interpolated trilinearly at the tail nodes
                                 (see gammax_model_predict_nodes_pooled) */
    int32_t projection;       /* point-to-simplex distance in the key-0 pass (3D): 0 = every face
                                 a cell owns, without branches (Algorithm A2's Kernel 3, default);
                                 1 = Ju et al.'s recursion (Algorithm A1 step 4-b-i): each
                                 tetrahedron, then only the facets, edges and vertices its
                                 negative weights point to.  Same gamma up to rounding. */
    int32_t reserved[1];      /* must be 0 */
    const float *order_key;   /* GAMMAX_SORT_GIVEN: device array, one float per grid node in the
                                 doses' layout (negative keys and NaN count as 0); read by the
                                 map, so it must stay valid and unchanged until the map is
                                 complete.  Ignored by the other orders. */
} gammax_options_t;

typedef struct {
    uint64_t n_evaluated;     /* M: masked reference nodes */
    uint64_t n_pass;          /* nodes with gamma <= 1 */
    uint64_t n_borderline;    /* nodes with |gamma - 1| <= 1e-5 (their pass decision is precision-bound) */
    uint64_t n_fp64_tets;     /* tetrahedron projections redone in FP64 by the guard */
    uint64_t n_cells;         /* full grid cells evaluated by the search, summed over nodes */
    uint64_t n_tail;          /* nodes that walked past the key-0 cells */
    uint64_t n_guarded;       /* nodes redone because they met an ill-conditioned tetrahedron */
    double pass_rate;         /* n_pass / n_evaluated (NaN when n_evaluated == 0) */
    float max_gamma;          /* largest gamma found */
    float dose_max;           /* max(D_r) */
    float search_radius;      /* R = max gamma0 = max |DD| / dD over masked nodes (Algorithm A1 step 1) */
    int32_t table_len;        /* cells in the sorted table used by the search */
    float ms_prep;            /* timing = 1 only: dose max, mask, gamma0, compaction */
    float ms_table;           /*   cell table build (0 when the cached table was reused) */
    float ms_search;          /*   search over the key-0 cells of every node (Algorithm A2 step 6) */
    float ms_sort;            /*   sort of the nodes that walk further (step 3) */
    float ms_tail;            /*   their table walk (step 6) */
    float ms_guard;           /*   FP64-guarded redo of nodes that met an ill-conditioned
                                   tetrahedron (guarded precision, 3D), and the count reduction */
    uint64_t n_fallback;      /* learned radius: tail nodes not certified inside f * gamma_hat */
    float ms_cnn;             /* timing = 1 only: the network at the tail nodes (learned radius),
                                 between the key-0 pass and the sort */
    float ms_done;            /* gammax_batch only: time from the start of the batch until the
                                 last work item of this pair finished (device clock) */
    uint32_t long_walk_rows;  /* longest walk past the key-0 cells, in table rows, when above
                                 256 (else 0).  The next map on the same context then uses
                                 wider lane groups for its tail (automatic tail_lanes only). */
} gammax_result_t;

typedef struct gammax_ctx gammax_ctx_t;

/* Fill `opt` with the defaults: no sort, guarded FP32, cond_threshold 1e6, no timing,
 * automatic tail lanes, plain radius, radius_factor 1.1. */
void gammax_options_default(gammax_options_t *opt);

/* Create a context bound to HIP device `device`.  *ctx receives the handle. */
gammax_status_t gammax_ctx_create(int device, gammax_ctx_t **ctx);

/* Release the context and everything it allocated.  NULL is accepted. */
gammax_status_t gammax_ctx_destroy(gammax_ctx_t *ctx);

/*
 * Gamma map of one dose pair (Algorithm A2 steps 2-7 on device memory).
 *   ref_dev, eval_dev : N = prod(shape) floats each (device).
 *   gamma_dev         : N floats (device, caller-owned) receive gamma; -1 marks nodes that
 *                       are not evaluated.  May not alias the inputs.
 *   opt               : NULL for the defaults.
 *   result            : host struct, required; filled on GAMMAX_OK.
 * Synchronises `stream` (the search radius and the counts come back to the host).
 */
gammax_status_t gammax_map(gammax_ctx_t *ctx, const gammax_problem_t *problem,
                           const gammax_options_t *opt, const float *ref_dev,
                           const float *eval_dev, float *gamma_dev, gammax_result_t *result,
                           void *stream);

/* Maps that may be in flight at once on one context (gammax_map_async). */
#define GAMMAX_ASYNC_SLOTS 64

/*
 * Queue one gamma map (the computation of gammax_map) without waiting for it, for callers
 * that issue maps back to back and collect the results afterwards: the host's launch work
 * for the next map then overlaps the GPU's work on this one.
 *   Arguments as in gammax_map, except: options->timing must be 0 (GAMMAX_E_PARAM), and
 *   *ticket receives a nonzero handle for gammax_map_wait.
 *   The doses, gamma and options->model must stay valid and the doses unchanged until
 *   gammax_map_wait returns for this ticket; gamma is complete after it returns.
 *   When the context has no cell table for this geometry yet, the map runs to completion
 *   inside this call (as gammax_map does) and the wait only returns its result.
 *   At most GAMMAX_ASYNC_SLOTS maps may be queued and not collected (GAMMAX_E_PARAM).
 *   Maps on one context run in issue order on their streams; give every map of a context
 *   the same stream (they share the context's workspace).
 */
gammax_status_t gammax_map_async(gammax_ctx_t *ctx, const gammax_problem_t *problem,
                                 const gammax_options_t *opt, const float *ref_dev,
                                 const float *eval_dev, float *gamma_dev, uint64_t *ticket,
                                 void *stream);

/*
 * Wait for a map queued by gammax_map_async and fill `result` (as gammax_map does).  Each
 * ticket is collected once; a second wait returns GAMMAX_E_PARAM.  Dose errors
 * (GAMMAX_E_NONFINITE, GAMMAX_E_DOSE) are reported here.  If the map's search radius
 * outgrew the cached cell table, the map runs again here, synchronously, on a larger table
 * (the doses must still hold the same values), and gamma is rewritten.
 */
gammax_status_t gammax_map_wait(gammax_ctx_t *ctx, uint64_t ticket, gammax_result_t *result);

/*
 * Gamma maps of n dose pairs in one call (the computation of gammax_map for each).  Pair i
 * uses a context of its own, kept by `ctx` for later calls at the same index (its cell
 * table, captured graph and workspace stay cached: a repeated batch replays), and the
 * pairs are queued round-robin on `stream` and three internal streams, so small maps run
 * beside large ones.  The maps start after the work queued on `stream` before the call, and later work
 * on `stream` follows them; the call returns when every map is complete.
 *   problems/refs/evals/gammas/results: n entries each; buffers as in gammax_map.
 *   opt: NULL for the defaults; timing must be 0.
 * On an error the status of the first failing pair is returned and gammax_last_error names
 * the pair; the maps already queued are completed first.
 */
gammax_status_t gammax_map_many(gammax_ctx_t *ctx, int32_t n, const gammax_problem_t *problems,
                                const float *const *refs_dev, const float *const *evals_dev,
                                float *const *gammas_dev, const gammax_options_t *opt,
                                gammax_result_t *results, void *stream);

/* An evaluation grid of its own (axis-aligned): shape and spacing slowest axis first, and the
 * position of its node 0 in the reference grid's frame (reference node k sits at
 * k * spacing_mm), in mm. */
typedef struct {
    int64_t shape[3];
    double spacing_mm[3];
    double origin_mm[3];
} gammax_grid_t;

/*
 * Gamma map with the evaluation dose on a grid of its own (not in the paper, which compares
 * doses on one grid; Eq. (1) unchanged, with the evaluation surface built over eval_grid).
 * 2D or 3D (eval_grid uses its first ndim entries).  problem: the reference grid and the
 * criteria; eval_dev: prod(eval_grid->shape) floats.  A 2D map runs as the 3D map of the
 * pair extruded to two layers (the Kuhn interpolant of a dose constant along the added axis
 * is the 2D interpolant, so the result is the 2D gamma), in context workspace.  A masked reference node inside the evaluation grid's closed box is evaluated;
 * the others get gamma = -1.  Each node walks a table of evaluation cells sorted by a key
 * that bounds the distance from below for any node position inside its holding cell, from
 * the nearest vertex of that cell.  Options: precision (FP32, guarded, FP64), tail_lanes
 * (0 = 16, or 8, 16, 32, 64 lanes per node), cond_threshold; the plain radius and no sort
 * only (others: GAMMAX_E_PARAM).  Result: counts, max gamma, dose max, search radius (the
 * largest first bound) and table length.  Synchronises `stream`.
 */
gammax_status_t gammax_map_grids(gammax_ctx_t *ctx, const gammax_problem_t *problem,
                                 const gammax_grid_t *eval_grid, const float *ref_dev,
                                 const float *eval_dev, float *gamma_dev, const gammax_options_t *opt,
                                 gammax_result_t *result, void *stream);

/*
 * The problem statement as a flat call (Sec. 2.1): gamma and pass rate of one dose pair
 * with the default options on a library-owned context for the current device.
 * shape/spacing_mm hold ndim entries each (slowest axis first); norm is gammax_norm_t.
 * pass_rate may be NULL.  Not thread-safe.
 */
gammax_status_t gamma_map(const float *ref_dose, const float *eval_dose, int32_t ndim,
                          const int64_t *shape, const double *spacing_mm, double dd,
                          double dta_mm, double dose_threshold, int32_t norm, float *gamma,
                          double *pass_rate, void *stream);

/*
 * Stable ascending sort of n (key, value) pairs of uint32 in place on the device: the
 * LDS radix sort used for the DD sort (Algorithm A2 step 3) and for the cell table
 * (step 5); up to 4096 pairs, the one-workgroup rank sort used for short tails.  Equal
 * keys keep their input order.
 */
gammax_status_t gammax_sort_pairs(gammax_ctx_t *ctx, uint32_t *keys_dev, uint32_t *vals_dev,
                                  int64_t n, void *stream);

/*
 * The radially sorted cell table (Algorithm A1 steps 2-3, Algorithm A2 steps 4-5).
 * Lists every cell offset a (lower corner relative to the reference node, slowest axis
 * first) that can hold a grid cell of `shape` and whose key
 *     key(a)^2 = sum_i (s_i * max(0, a_i, -a_i - 1))^2,  s_i = spacing_i / DTA,
 * is < radius^2, in ascending key order (ties: slowest axis, then the others, ascending).
 * key2_dev receives key(a)^2 rounded toward -inf to float; offs_dev receives 3 int32 per
 * entry (2D: a_y, a_x, 0).  cap is the capacity of both buffers in entries; *len receives
 * the entry count, or GAMMAX_E_RADIUS is returned when it would exceed cap.
 * Synchronises `stream`.
 */
gammax_status_t gammax_build_table(gammax_ctx_t *ctx, int32_t ndim, const int64_t *shape,
                                   const double *spacing_over_dta, double radius,
                                   float *key2_dev, int32_t *offs_dev, int64_t cap,
                                   int64_t *len, void *stream);

/*
 * Pass-rate counts of a gamma map (n floats, device): counts[0] = nodes with gamma >= 0
 * (evaluated), counts[1] = gamma <= 1, counts[2] = |gamma - 1| <= 1e-5.  Synchronises.
 */
gammax_status_t gammax_pass_count(gammax_ctx_t *ctx, const float *gamma_dev, int64_t n,
                                  uint64_t *counts, void *stream);

/*
 * ---- Learned search radius (an addition around the paper's method) ----------------------
 *
 * A small 3D CNN predicts y = log(gamma + 0.01) at every node from the 9x9x9 neighbourhood
 * of two features, f0 = D_r / max D_r and f1 = (D_e - D_r) / (DD * max D_r) (global dD),
 * zero outside the grid.  Four valid 3x3x3 convolutions with channels 2 -> 16 -> 16 ->
 * 16 -> 1, ReLU after the first three, over the features padded by 4 nodes.  bf16
 * operands on the matrix cores, FP32 accumulation and biases, bf16 hidden activations.
 * The prediction only orders the search and bounds its first attempt; every gamma the
 * library returns is still the exact search result.
 *
 * Parameters: GAMMAX_MODEL_NPARAM floats, per layer W[co][ci][dz][dy][dx] then b[co].
 */
#define GAMMAX_MODEL_NPARAM 15169

typedef struct {
    float lr;       /* Adam step size */
    float beta1;    /* 0.9 */
    float beta2;    /* 0.999 */
    float eps;      /* 1e-8 */
} gammax_adam_t;

/* Create a model on HIP device `device` from GAMMAX_MODEL_NPARAM host floats (copied). */
gammax_status_t gammax_model_create(int device, const float *params, gammax_model_t **model);

/* Release the model.  NULL is accepted. */
gammax_status_t gammax_model_destroy(gammax_model_t *model);

/* Copy the FP32 parameters and/or the gradient of the last training step (each
 * GAMMAX_MODEL_NPARAM host floats; either pointer may be NULL, not both).  Synchronises. */
gammax_status_t gammax_model_get_params(gammax_model_t *model, float *params, float *grad);

/* Detail of the last failure of a model call; never NULL. */
const char *gammax_model_last_error(const gammax_model_t *model);

/*
 * Checkpoint of a model: its FP32 parameters and the Adam state of its training steps, so
 * that training resumes where it stopped (gammax_model_train_step continues the bias
 * correction from the stored step count).  File layout: one line of JSON ending in '\n',
 *     {"format": "gammax-model", "version": 1, "nparam": 15169, "adam_step": S,
 *      "arrays": ["params", "adam_m", "adam_v"], "dtype": "float32-le"}
 * then the three arrays of GAMMAX_MODEL_NPARAM little-endian float32 each, in that order
 * (parameters in the flat layout above, then Adam's first and second moment estimates).
 * save: writes `path` (replaced if it exists); synchronises the model's device.
 *   GAMMAX_E_MODEL when the file cannot be written.
 * load: creates a model on HIP device `device` from such a file (*model receives it, or
 *   NULL on failure).  GAMMAX_E_MODEL when the file cannot be read, its header is not this
 *   format and version or holds another parameter count, the data is short or too long, or
 *   a stored value is not finite.
 */
gammax_status_t gammax_model_save(const gammax_model_t *model, const char *path);
gammax_status_t gammax_model_load(int device, const char *path, gammax_model_t **model);

/*
 * Input features of one dose pair on the grid padded by 4 nodes: (nz+8) x (ny+8) x (nx+8)
 * nodes of 2 bf16 each (uint16 bit patterns, channel fastest), device memory.  3D only.
 * Uses the context's dose maximum pass.  Synchronises.
 */
gammax_status_t gammax_model_features(gammax_ctx_t *ctx, const gammax_problem_t *problem,
                                      const float *ref_dev, const float *eval_dev,
                                      uint16_t *feat_dev, void *stream);

/*
 * Prediction y = log(gamma_hat + 0.01) at every node of one dose pair (N floats, device).
 * 3D only.  Synchronises.
 */
gammax_status_t gammax_model_predict(gammax_ctx_t *ctx, gammax_model_t *model,
                                     const gammax_problem_t *problem, const float *ref_dev,
                                     const float *eval_dev, float *y_dev, void *stream);

/*
 * Prediction at listed nodes only: y_dev[i] = log(gamma_hat + 0.01) at flat node index
 * nodes_dev[i] (i < n), each from its own 9x9x9 patch (the values the whole-grid
 * prediction gives there, up to the order of the last layer's FP32 sum).  This is how the
 * learned radius is evaluated inside gammax_map: only at the nodes that walk past the
 * key-0 cells.  3D only.  Synchronises.
 */
gammax_status_t gammax_model_predict_nodes(gammax_ctx_t *ctx, gammax_model_t *model,
                                           const gammax_problem_t *problem, const float *ref_dev,
                                           const float *eval_dev, const uint32_t *nodes_dev, int64_t n,
                                           float *y_dev, void *stream);

/*
 * Prediction at listed nodes of a grid finer than the model's training grid (the network
 * input is not a quantity of the paper; the pooling keeps the network at the spacing it
 * was trained on).  The pair is average-pooled 2x2x2 onto the coarse grid ceil(n / 2) per
 * axis (coarse node c takes the mean of the fine nodes 2c, 2c + 1 per axis that exist), the
 * features use the fine grid's max reference dose, the network runs on the whole coarse
 * grid (as gammax_model_predict), and at each listed fine node p the coarse values
 * gamma_hat + 0.01 = exp(y) are interpolated trilinearly at coarse position (p - 1/2) / 2
 * per axis (clamped to the coarse grid): y_dev[i] = log of that value.  This is what
 * gammax_map evaluates with options cnn_pool = 2.  Arguments as gammax_model_predict_nodes;
 * the workspace (coarse features and activations) belongs to the context.  Synchronises.
 */
gammax_status_t gammax_model_predict_nodes_pooled(gammax_ctx_t *ctx, gammax_model_t *model,
                                                  const gammax_problem_t *problem, const float *ref_dev,
                                                  const float *eval_dev, const uint32_t *nodes_dev, int64_t n,
                                                  float *y_dev, void *stream);

/*
 * Forward pass over nvol crops: feat_dev holds nvol volumes of (c0+8) x (c1+8) x (c2+8)
 * feature nodes (2 bf16 each), y_dev receives nvol x c0 x c1 x c2 floats.  Synchronises.
 */
gammax_status_t gammax_model_forward(gammax_model_t *model, int32_t nvol, const int64_t *crop,
                                     const uint16_t *feat_dev, float *y_dev, void *stream);

/*
 * One training step on nvol crops: features as in gammax_model_forward, gamma_dev holds
 * nvol x c0 x c1 x c2 labels (gamma >= 0 marks a node that counts; others are ignored).
 * Loss = mean over counted nodes of (y - log(gamma + 0.01))^2.  Computes the gradient
 * (readable with gammax_model_get_params), takes one Adam step on the FP32 parameters
 * and returns the loss before the step in *loss (may be NULL).  Synchronises.
 */
gammax_status_t gammax_model_train_step(gammax_model_t *model, int32_t nvol, const int64_t *crop,
                                        const uint16_t *feat_dev, const float *gamma_dev,
                                        const gammax_adam_t *adam, double *loss, void *stream);

/*
 * ---- Batches of dose pairs ------------------------------------------------------------
 *
 * Gamma maps of n pairs of any mix of dimensionality, grid, spacing, criteria and
 * normalisation, with one set of options, as one launch of a HIP graph captured on one
 * stream (replayed when the same batch comes again).  Each pair index keeps a context of its own inside
 * `ctx` (its cell table, workspace and scalars); a pair met for the first time at its index
 * (or with a new geometry) first runs its map alone, which builds its table.  The graph
 * holds, in order: every pair's compaction (dose maximum, mask, gamma0, ordered node list);
 * one launch of the key-0 pass over every pair's nodes, one workgroup per (pair, block of
 * 256 nodes), the blocks in cost order (3D pairs first, larger pairs first); then every
 * pair's own pipeline after the key-0 pass (the network at its tail nodes when learned, tail
 * sort, tail walk and fallback, FP64 guard, count reduction).
 *   problems[i], refs[i], evals[i], gammas[i]: pair i, as in gammax_map.
 *   opt: NULL for the defaults; timing, the given order, projection 1 and one lane per cell
 *   are refused (GAMMAX_E_PARAM).  The learned radius applies to the 3D pairs.
 *   results[i]: filled on GAMMAX_OK; ms_done = device time from the start of the batch until
 *   the end of pair i's pipeline.
 * With opt->autotune = 1 (and tail_lanes 0), each shape class (dimensionality, size,
 * criteria, spacing) met for the first time has its tail layout (automatic, 8, 16, 32 or 64
 * lanes per node) chosen by timing the tail walk of the first pair of the class with each
 * (that pair's own map with phase events), and the choice is kept in the context
 * (gammax_tune_save/load).  A pair whose search radius outgrew its cached table is
 * run again on its own, on a larger table (the next batch recaptures the graph).
 * A device-side error of any pair (non-finite dose, no positive dose) fails the batch;
 * gammax_last_error names the pair.  Synchronises `stream`.
 */
gammax_status_t gammax_batch(gammax_ctx_t *ctx, int32_t n, const gammax_problem_t *problems,
                             const float *const *refs, const float *const *evals, float *const *gammas,
                             const gammax_options_t *opt, gammax_result_t *results, void *stream);

/* Write / read the context's tuned tail layouts (one text line per shape class). */
gammax_status_t gammax_tune_save(const gammax_ctx_t *ctx, const char *path);
gammax_status_t gammax_tune_load(gammax_ctx_t *ctx, const char *path);

/*
 * ---- The map without device allocations -------------------------------------------------
 *
 * For callers that cannot allocate device memory (code that must not call hipMalloc, tight
 * serving loops, harnesses that forbid allocation).  The computation of gammax_map; every
 * buffer beyond the caller's doses and gamma lives in one fixed array of
 * GAMMAX_NOALLOC_SCRATCH_BYTES bytes of device memory inside the library, which each GPU
 * the library runs on holds from the library's load until the process ends.  No context:
 * the call uses the current HIP device and `stream`, allocates nothing, builds the cell
 * table for this map's radius in that array, and synchronises `stream` (three times: after
 * the compaction, after the table count, at the end).
 *   Limits: at most GAMMAX_NOALLOC_MAX_NODES grid nodes (GAMMAX_E_SHAPE beyond), a cell
 *   table of at most GAMMAX_NOALLOC_MAX_TABLE rows and a candidate box of at most twice
 *   that (GAMMAX_E_RADIUS beyond).
 *   opt: NULL for the defaults; timing, a model (learned radius or predicted order), the
 *   given order, autotune and cnn_pool are refused (GAMMAX_E_PARAM).
 *   result: as gammax_map, except table_len (the rows of this call's own table) and the
 *   timing fields (0).
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (from
 * several host threads or streams) race and give wrong results; serialise them.
 */
#define GAMMAX_NOALLOC_MAX_NODES 2097152
#define GAMMAX_NOALLOC_MAX_TABLE 262144
#define GAMMAX_NOALLOC_SCRATCH_BYTES 104857600
gammax_status_t gammax_map_noalloc(const gammax_problem_t *problem, const gammax_options_t *opt,
                                   const float *ref_dev, const float *eval_dev, float *gamma_dev,
                                   gammax_result_t *result, void *stream);

/* Static description of a status code. */
const char *gammax_status_string(gammax_status_t status);

/* Detail of the last failure on this context (HIP error text etc.); never NULL. */
const char *gammax_last_error(const gammax_ctx_t *ctx);

#ifdef __cplusplus
}
#endif
#endif /* GAMMAX_H */
