// Internal declarations shared by the HIP translation units of libgammax.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gammax {

// Device-resident scalars of one gamma_map call.  One copy lives in device memory; the
// host reads it back once the search has finished.
struct Scalars {
    uint32_t dmax_ord;      // max D_r as an order-preserving uint32 (see float_to_ord)
    uint32_t r2_bits;       // max gamma0^2 over masked nodes (non-negative float bits)
    uint32_t n_masked;      // M
    uint32_t flags;         // FLAG_*
    uint32_t maxg2_bits;    // max gamma^2 found (non-negative float bits)
    float thr_val;          // fl32(fl32(threshold) * max D_r): mask is D_r >= thr_val
    float inv_dd;           // 1 / fl32(DD * max D_r) (global normalisation)
    uint32_t n_guard;       // nodes queued for the FP64-guarded pass
    unsigned long long n_pass;
    unsigned long long n_border;
    unsigned long long n_fp64;
    unsigned long long n_cells;
};

enum : uint32_t { FLAG_NONFINITE = 1u };

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

// Order-preserving map of floats onto uint32 (for atomicMax over signed values).
__host__ __device__ inline uint32_t float_to_ord(float f) {
    uint32_t u = f2u(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float ord_to_float(uint32_t o) {
    uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return u2f(u);
}

// gamma0^2 of a node, the upper bound every search starts from (Algorithm A1 step 4a).
// The same expression is used by the compaction and by the search so that both see the
// same bits.
__device__ __forceinline__ float node_inv_dd(float dr, float inv_dd_global, float dd, int local) {
    return local ? 1.0f / (dd * dr) : inv_dd_global;
}
__device__ __forceinline__ float gamma0_sq(float de, float dr, float inv_dd) {
    float g = (de - dr) * inv_dd;
    return g * g;
}

// ---- launchers (each defined next to its kernels) -------------------------------------

struct PrepArgs {
    const float* ref;
    const float* ev;
    float* gamma;
    int64_t n;
    float thr;          // fl32(threshold)
    float dd;           // fl32(DD)
    int local;
    Scalars* sc;
    uint32_t* blockcnt; // one per prep tile
    uint32_t* keys;     // M entries: gamma0^2 bits
    uint32_t* vals;     // M entries: node index
};

constexpr int PREP_THREADS = 256;
constexpr int PREP_ITEMS = 16;
constexpr int PREP_TILE = PREP_THREADS * PREP_ITEMS;

hipError_t launch_init_scalars(Scalars* sc, hipStream_t s);
hipError_t launch_dose_max(const float* ref, const float* ev, int64_t n, Scalars* sc, hipStream_t s);
hipError_t launch_prep(const PrepArgs& a, hipStream_t s);  // count, scan, emit
hipError_t launch_pass_count(const float* gamma, int64_t n, unsigned long long* counts3, hipStream_t s);

// LDS radix sort of (key, value) uint32 pairs.  tmp_* hold n entries each; hist needs
// sort_hist_words(n) words.  The sorted result ends in keys/vals.
int64_t sort_hist_words(int64_t n);
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals,
                            int64_t n, uint32_t* hist, hipStream_t s);

struct TableGeom {
    int ndim;
    int64_t shape[3];   // slowest first
    double s[3];        // spacing / DTA, slowest first
    double r2_cap;      // entries with key^2 < r2_cap
    int64_t lo[3], ext[3];  // candidate box per axis (slowest first)
    int64_t box;        // prod(ext)
};
void table_box(TableGeom& g);
// Fill keys (rounded-down key^2 bits, or 0xFFFFFFFF when key^2 >= r2_cap) and values
// (box index) for every candidate, counting the kept ones into *count.
hipError_t launch_table_gen(const TableGeom& g, uint32_t* keys, uint32_t* vals, uint32_t* count,
                            hipStream_t s);
// Rows of the first n sorted candidates.
hipError_t launch_table_rows(const TableGeom& g, const uint32_t* vals, int64_t n, TabEntry* rows,
                             hipStream_t s);
hipError_t launch_table_export(const TabEntry* rows, int64_t n, int ndim, float* key2, int32_t* offs,
                               hipStream_t s);

struct SearchArgs {
    const float* ref;
    const float* ev;
    float* gamma;
    const uint32_t* order;   // node indices in work order
    uint32_t* guard_list;    // nodes that met an ill-conditioned tetrahedron (capacity M)
    const Scalars* sc_in;    // n_masked
    Scalars* sc;             // counters
    const TabEntry* tab;
    int tab_len;
    int nx, ny, nz;          // nz = 1 in 2D
    float dd;                // fl32(DD); local: dD = DD * D_r
    double dd64;             // DD in double for the FP64 paths
    int local;
    float s2x, s2y, s2z;     // s_i^2, s_i = spacing_i / DTA
    float den_guard;         // FP64 re-projection when the tetrahedron's Den exceeds this
    double sx, sy, sz;       // s_i in double for the FP64 paths
};
// Main search pass over the M nodes in work order.
hipError_t launch_search(const SearchArgs& a, int ndim, int precision, uint32_t max_items,
                         hipStream_t s);
// Guarded precision only: nodes that met an ill-conditioned tetrahedron, again with FP64
// re-projection (grid-stride over the device-side list; returns at once when it is empty).
hipError_t launch_search_guard(const SearchArgs& a, int ndim, int precision, hipStream_t s);

}  // namespace gammax
