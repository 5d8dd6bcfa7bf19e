// Internal declarations shared by the HIP translation units of libgammax.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gammax {

// Device-resident scalars of one gamma map.  The host reads them back after the
// compaction (M, R) and after the search (counts).
struct Scalars {
    uint32_t dmax_ord;      // max D_r as an order-preserving uint32 (see float_to_ord)
    uint32_t r2_bits;       // max gamma0^2 over masked nodes (non-negative float bits)
    uint32_t n_masked;      // M
    uint32_t flags;         // FLAG_*
    float thr_val;          // fl32(fl32(threshold) * max D_r): mask is D_r >= thr_val
    float inv_dd;           // 1 / fl32(DD * max D_r) (global normalisation)
    uint32_t n_tail;        // nodes whose walk continues past the zero-key cells
    uint32_t n_guard;       // nodes queued for the FP64-guarded pass
    uint32_t maxg2_bits;    // max gamma^2 found (non-negative float bits)
    uint32_t n_fallback;    // learned radius: tail nodes not certified inside 1.1 * gamma_hat
    uint32_t sort_overflow; // the one-workgroup tail sort met a longer tail (left unsorted)
    uint32_t long_rows;     // longest tail walk in table rows, when above LONG_WALK_ROWS (else 0)
    uint32_t n_fallback_inline;   // learned radius, short tail: nodes the prediction would not certify
    uint32_t reserved;
    unsigned long long n_pass;
    unsigned long long n_border;
    unsigned long long n_fp64;
    unsigned long long n_cells;
};

enum : uint32_t { FLAG_NONFINITE = 1u, FLAG_TABLE_SHORT = 2u };
// A tail walk longer than this many table rows is recorded in Scalars::long_rows.
constexpr uint32_t LONG_WALK_ROWS = 256;

// Per-block partial counts of a search launch; reduced by one finishing block (no
// contended atomics on a single address).
struct BlockSums {
    unsigned long long pass, border, fp64, cells;
    uint32_t maxg2, pad;
};
constexpr int SUM_BINS = 256;   // partial-count slots of one gamma map (zeroed by the prep)

// One row of the sorted cell table.  Everything that depends only on the cell offset
// and the normalised spacing is precomputed here, so a wave reads it with one scalar
// load.  Axis letters: x = fastest array axis, y, z = slowest (3D).
//   key2   : key(a)^2 rounded down to float
//   a*     : cell offset (lower corner minus reference node), voxels
//   px..pz : s_i^2 a_i^2 (squared spatial distance components to the lower corner)
//   v*     : spatial residual of a multi-axis chain block B (the part of
//            sum_{i in B} s_i^2 a_i^2 that a common parameter t cannot remove):
//            v_B = sum_{i<j in B} s_i^2 s_j^2 (a_i - a_j)^2 / sum_{i in B} s_i^2
//   m*     : foot parameter of block B: mu_B = sum_{i in B} s_i^2 a_i / sum_{i in B} s_i^2
struct alignas(16) TabEntry {
    float key2;
    int32_t ax, ay, az;
    float px, py, pz, vxy;
    float vxz, vyz, vxyz, mxy;
    float mxz, myz, mxyz, pad;
};
static_assert(sizeof(TabEntry) == 64, "table entry is one 64-byte row");

__host__ __device__ inline uint32_t f2u(float f) { return __builtin_bit_cast(uint32_t, f); }
__host__ __device__ inline float u2f(uint32_t u) { return __builtin_bit_cast(float, u); }

// Order-preserving map of floats onto uint32 (max over signed values).
__host__ __device__ inline uint32_t float_to_ord(float f) {
    uint32_t u = f2u(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float ord_to_float(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return u2f(u);
}

// gamma0^2 of a node, the upper bound every search starts from (Algorithm A1 step 4a).
// Compaction and search use this one expression, so both see the same bits.
__device__ __forceinline__ float node_inv_dd(float dr, float inv_dd_global, float dd, int local) {
    return local ? 1.0f / (dd * dr) : inv_dd_global;
}
__device__ __forceinline__ float gamma0_sq(float de, float dr, float inv_dd) {
    float g = (de - dr) * inv_dd;
    return g * g;
}

// ---- prep: dose max, mask, gamma0, ordered compaction ---------------------------------

constexpr int PREP_THREADS = 256;
constexpr int PREP_ITEMS = 4;
constexpr int PREP_TILE = PREP_THREADS * PREP_ITEMS;
constexpr int MAX_BLOCKS = 1024;   // blocks of the grid-stride dose-max reduction

struct PrepArgs {
    const float* ref;
    const float* ev;
    float* gamma;
    int64_t n;
    float thr;          // fl32(threshold)
    float dd;           // fl32(DD)
    int local;
    Scalars* sc;
    uint32_t* part;     // 2 * MAX_BLOCKS words: dose-max partials and non-finite flags
    uint32_t* blockcnt; // one per prep tile: masked count
    uint32_t* super;    // 2 * n_super: masked count and max gamma0^2 bits per group of tiles
    int ntiles;         // prep tiles (prep_tiles(n))
    int super_shift;    // a group holds 2^super_shift consecutive tiles
    int n_super;
    uint32_t* nodes;    // M entries: masked node indices in grid order
    BlockSums* sums;    // SUM_BINS partial-count slots of the search, zeroed here
    unsigned long long* mbits;   // mask bits, one word per 64 nodes of the prep tiles
};

int64_t prep_tiles(int64_t n);
// Tile groups of the compaction: 2^shift >= sqrt(tiles) tiles per group; words = the
// tile counts, two words per group, then the mask bits (two words per 64 nodes).
void prep_groups(int64_t n, int* shift, int* n_super);
int64_t prep_words(int64_t n);
// Offset (32-bit words, even) of the mask bits within the prep words: after the tile counts
// and the group words.
int64_t prep_mbits_offset(int64_t n);
hipError_t launch_prep(const PrepArgs& a, hipStream_t s);
// Only the dose maximum, the finiteness flag, the threshold value and the global 1/dD
// (uses ref, ev, n, thr, dd, sc, part).
hipError_t launch_dose_scalars(const PrepArgs& a, hipStream_t s);
hipError_t launch_pass_count(const float* gamma, int64_t n, unsigned long long* counts3, hipStream_t s);

// ---- sort --------------------------------------------------------------------------------

// LDS radix sort of (key, value) uint32 pairs.  n_dev (optional) holds the element count
// on the device, at most n_max; without it n_max is the count.  tmp_* hold n_max entries;
// hist needs sort_hist_words(n_max) words.  The result ends in keys/vals.
int64_t sort_hist_words(int64_t n_max);
// Stable rank sort for lists of at most SMALL_SORT_CAP pairs in two launches (count on the
// device; tmp_* hold SMALL_SORT_CAP entries); a longer list is left unsorted and *overflow
// set to 1.
constexpr int SMALL_SORT_CAP = 4096;
hipError_t sort_pairs_small(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals,
                            const uint32_t* n_dev, uint32_t* overflow, hipStream_t s);
// The same rank sort of a list whose values are its positions 0..n-1: order[] receives the
// positions in stable key order (one launch; the keys stay where they are).
// Sort keys of the queued tail nodes from a caller's per-node key: key[i] = the bits of
// max(given[nodes[i]], 0) (NaN as 0) for i < *count.
hipError_t launch_given_keys(const uint32_t* nodes, const uint32_t* count, const float* given, uint32_t* key,
                             hipStream_t s);
hipError_t sort_order_small(const uint32_t* keys, uint32_t* order, const uint32_t* n_dev, uint32_t* overflow,
                            hipStream_t s);
// Stable LSD radix sort of (key, value) pairs by key bits [low_bit, 32), 8 bits a pass:
// low_bit 0 sorts whole keys; 16 sorts by the top half (2 passes), which for non-negative
// float keys orders by value to 7 mantissa bits and keeps the input order within a bucket.
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals,
                            int64_t n_max, const uint32_t* n_dev, uint32_t* hist, hipStream_t s, int low_bit = 0);

// ---- cell table --------------------------------------------------------------------------

struct TableGeom {
    int ndim;
    int64_t shape[3];   // slowest first
    double s[3];        // spacing / DTA, slowest first
    double r2_cap;      // entries with key^2 < r2_cap
    int lower = 0;      // 1: the key is the lower bound over every node position inside the
                        // holding cell, sum_i (s_i max(0, |a_i| - 1))^2 (two grids)
    int64_t lo[3], ext[3];  // candidate box per axis (slowest first)
    int64_t box;        // prod(ext)
};
void table_box(TableGeom& g);
hipError_t launch_table_gen(const TableGeom& g, uint32_t* keys, uint32_t* vals, uint32_t* count,
                            hipStream_t s);
hipError_t launch_table_rows(const TableGeom& g, const uint32_t* vals, int64_t n, TabEntry* rows,
                             hipStream_t s);
hipError_t launch_table_export(const TabEntry* rows, int64_t n, int ndim, float* key2, int32_t* offs,
                               hipStream_t s);
// The same row on the host (double, rounded to float like the device rows); used for the
// zero-key cells, whose constants the first search pass takes as kernel arguments.
void table_row_host(int ndim, const double s[3], int az, int ay, int ax, TabEntry* out);

// ---- search ------------------------------------------------------------------------------

struct SearchArgs {
    const float* ref;
    const float* ev;
    float* gamma;
    Scalars* sc;             // inputs n_masked, inv_dd, dmax; counters n_tail, n_guard
    const TabEntry* tab;
    int tab_len;
    int nx, ny, nz;          // nz = 1 in 2D
    float dd;                // fl32(DD); local: dD = DD * D_r
    double dd64;             // DD in double for the FP64 paths
    int local;
    float s2x, s2y, s2z;     // s_i^2, s_i = spacing_i / DTA
    float inv_s2[7];         // FP32 1 / sigma^2 of the chain blocks x, y, z, xy, xz, yz, xyz
                             // (sigma_B^2 = sum over B of s_i^2; the z terms are 0 in 2D)
    float den_guard;         // FP64 re-projection when a tetrahedron's Den exceeds this
    double sx, sy, sz;       // s_i in double for the FP64 paths
    float k1;                // key^2 of the first table row after the zero-key cells (+inf: none)
    float r2_cap;            // the table holds every cell with key^2 < r2_cap
    int tail_key;            // key of the tail sort: 0 = gamma0^2 (DD sort), 1 = bound after the
                             // key-0 cells, 2 = predicted gamma (learned ordering)
    const float* yhat;       // learned radius: log(gamma_hat + 0.01) per tail item, or null
    float spec_factor;       // the speculative walk stops at key >= spec_factor * gamma_hat
    // work lists
    const uint32_t* nodes;   // masked nodes in grid order (M)
    uint32_t* tail_node;     // tail: node index
    uint32_t* tail_f;        // tail: gamma^2 bound after the zero-key cells (float bits)
    uint32_t* tail_key_arr;  // tail: sort key
    uint32_t* tail_pos;      // tail: position (sort payload)
    uint32_t* guard_list;    // nodes that met an ill-conditioned tetrahedron
    uint32_t* fb_list;       // learned radius: tail items to finish with the plain walk
    BlockSums* sums;         // per-block partial counts
};

struct ZeroGeo {
    TabEntry row[8];         // the 2^d zero-key cells in table order
};

// The whole search on `s`: zero-key pass over all M nodes (grid order), sort of the tail,
// tail walk from the first non-zero key, FP64-guarded pass (precision 1), count reduction.
// precision: 0 FP32, 1 guarded FP32, 2 FP64 (one walk over all nodes).
struct SearchPlan {
    int ndim, precision;
    int tail_lanes;          // lanes per node in the tail walk: 1 (one lane per node) or 8..64
    int tail_min_lanes;      // automatic tail lanes (tail_lanes 0): at least this many (0: 8)
    int zero_lanes;          // pass A: 1 = one lane per cell, 0 = one lane per node
    int projection;          // pass A in 3D: 0 = all faces a cell owns, 1 = Ju's recursion
    int skip_zero;           // 1: the key-0 pass was queued elsewhere (a batch's launch over all pairs)
    int spec;                // 1: speculative tail walk inside spec_factor * gamma_hat, then the
                             //    plain walk for the nodes it could not certify; 3: a short tail
                             //    (groups of 64 lanes), walked with the plain bound, the nodes
                             //    the prediction would not certify counted as fallbacks
    // optional: queued after the key-0 pass, before the tail sort (the network at the tail
    // nodes writes yhat and, for the predicted order, the sort keys)
    hipError_t (*after_zero)(void* user, hipStream_t s);
    void* after_zero_user;
    uint32_t M;
    ZeroGeo zero;
    uint32_t* tmp_keys;      // sort scratch, M entries each
    uint32_t* tmp_vals;
    uint32_t* hist;          // sort_hist_words(M)
    int small_sort;          // sort the tail with the rank sort (expected to hold <= SMALL_SORT_CAP)
    hipEvent_t ev_shell_end; // optional: recorded after the zero-key pass
    hipEvent_t ev_sort_end;  // optional: recorded after the tail sort
    hipEvent_t ev_tail_end;  // optional: recorded after the tail walk
};
int64_t search_sums_needed(uint32_t M);
hipError_t launch_search(const SearchArgs& a, const SearchPlan& plan, hipStream_t s);

// ---- two grids: the evaluation dose on a grid of its own (3D) ---------------------------
//
// Reference node k sits at k * rh (mm, slowest axis first); evaluation node j at eo + j * eh.
// A masked reference node inside the evaluation grid's box is evaluated against the Kuhn
// surface of the evaluation grid; others get gamma = -1.
struct GridsArgs {
    const float* ref;
    const float* ev;
    float* gamma;
    int rn[3], en[3];          // shapes, slowest first
    double rh[3], eh[3], eo[3];
    double dta, dd;
    float thr;
    int local;
    float den_guard;
    Scalars* sc;               // dmax_ord, thr_val, inv_dd, n_masked (= nodes listed), r2_bits,
                               // n_guard, maxg2_bits, n_pass, n_border, n_cells, flags
    uint32_t* list;            // listed nodes
    float* f0;                 // their first bound (nearest vertex of the holding cell, dist^2)
    uint32_t* guard_list;      // nodes that met an ill-conditioned tetrahedron
    const TabEntry* tab;       // lower-key table of the evaluation grid
    int tab_len;
    float k1;                  // key^2 of the first row past the 27 key-0 cells
    uint32_t* tail_list;       // nodes the key-0 pass leaves for the walk (count: sc->n_tail)
    float* tail_f;             // and their bound so far
    uint32_t* part;            // MAX_BLOCKS words: per-block dose maxima (order-preserving bits)
};
// Dose maximum and finiteness, then the listing of the evaluated nodes with their first
// bound (and gamma = -1 everywhere else); sc must be zeroed before.
hipError_t launch_grids_prep(const GridsArgs& a, hipStream_t s);
// The walk of the listed nodes: precision 0 FP32, 1 FP32 with the guard (ill-conditioned
// nodes go to the guard list), 2 FP64; guard: walk the guard list in FP64 instead.
hipError_t launch_grids_walk(const GridsArgs& a, int precision, bool guard, int lanes, hipStream_t s);
// FP32 (precision 0, or 1 with the guard): the 27 key-0 cells of every listed node from its
// shared 4x4x4 neighbourhood, one lane per node; nodes not finished go to the tail list, and
// the walk of that list (tail = true) starts past the key-0 rows.
hipError_t launch_grids_zero(const GridsArgs& a, int precision, hipStream_t s);
hipError_t launch_grids_tail(const GridsArgs& a, int precision, int lanes, hipStream_t s);

// ---- batches of dose pairs -------------------------------------------------------------
//
// A batch runs each phase of the map as one launch over all its pairs: block b takes item
// b = (pair, block of that pair) and runs that pair's phase body exactly as the pair's own
// kernel would run that block.  The host lists the items of every launch; a pair's blocks
// are those its own launch would have (every grid is sized from the pair's node count, and
// the bodies read the device-side counts themselves).

struct BatchPair {
    SearchArgs sa;           // the pair's search arguments (those of its own pipeline)
    ZeroGeo zg;
    PrepArgs pa;             // its compaction arguments
    int ndim, guarded;       // guarded: FP32 with the FP64 guard (3D)
    int nbr;                 // blocks of its dose-maximum pass
    int first;               // first table row of its tail walk (2^d)
    int g_req;               // lanes per tail node (negative: automatic with that least width)
    int tail_blocks;         // grid-stride blocks of its tail walk
    int walk;                // 1: its table reaches past the key-0 rows
    int pad;
    uint32_t* seq;           // its map counter and pinned scalar ring (the publish)
    Scalars* ring;
    unsigned long long* done;  // its completion stamp (device clock)
};

// Blocks of the dose-maximum pass of an n-node pair.
int prep_reduce_blocks(int64_t n);
// Grid-stride blocks of the tail walk of a pair of at most m_bound nodes with lanes request g.
unsigned tail_grid_blocks(uint32_t m_bound, int g);
// Grid-stride blocks of the FP64 guard pass.
unsigned guard_grid_blocks();
// The compaction of every pair: dose maximum (items dm), then the count and the ordered
// emit of the masked nodes (items tiles: (pair, prep tile)).
hipError_t launch_batch_prep(const BatchPair* pairs, const uint2* dm, int n_dm, const uint2* tiles, int n_tiles,
                             hipStream_t s);
// The key-0 pass of every pair: items (pair, block of 256 nodes).
hipError_t launch_batch_key0(const BatchPair* pairs, const uint2* items, int n_items, hipStream_t s);
// The tail walk of every pair that has one: items (pair, tail block).
hipError_t launch_batch_tail(const BatchPair* pairs, const uint2* items, int n_items, hipStream_t s);
// Every pair's FP64 guard pass and count reduction (items (pair, guard block); one block for
// a pair without the guard), then its completion stamp.
hipError_t launch_batch_finish(const BatchPair* pairs, const uint2* items, int n_items, hipStream_t s);
// One thread writes the device's wall clock (for per-pair completion times).
hipError_t launch_stamp(unsigned long long* t, hipStream_t s);

}  // namespace gammax
