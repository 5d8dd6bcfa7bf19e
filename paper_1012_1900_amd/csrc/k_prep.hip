// Normalisation, mask, gamma0 and ordered compaction (Algorithm A2 step 2, "Kernel 1"),
// plus the stand-alone pass-rate reduction.
//
// Three launches, each a coalesced stream over the dose arrays; results cross blocks only
// at kernel boundaries or through atomic adds (a cross-block hand-over inside a kernel
// would need device-scope release fences, which write back the XCD's L2):
//   1. maximum and finiteness of D_r: one partial per block (block 0 also clears the
//      tile-group sums and the flags);
//   2. every block reduces those partials itself (a few KB from L2), derives the
//      threshold and the global 1/dD, then counts the masked nodes of its tile and their
//      max gamma0^2, checks D_e's finiteness, stores the tile's mask bits and count and
//      adds the count and the maximum into its tile group (about sqrt(tiles) / 8 tiles per
//      group, so no address sees many atomics); block 0 also stores the scalars and clears
//      the search counters;
//   3. ordered emit of the masked node indices from the mask bits: a block's first slot is
//      the sum of the groups before its own plus the tiles of its group before it; the
//      last block stores M and R^2.
// Each dose volume is read once by the compaction except D_r, read twice (its maximum sets
// the threshold that the mask needs); the emit reads one bit per node.
#include "internal.hpp"

namespace gammax {

namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
    return v;
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o);
    return v;
}

// Block-wide max and or over PREP_THREADS threads (result valid in every thread).
__device__ __forceinline__ void block_max_or(uint32_t& m, uint32_t& f) {
    __shared__ uint32_t s_m[PREP_THREADS / WAVE], s_f[PREP_THREADS / WAVE];
    m = wave_max_u32(m);
    f = __ballot(f != 0u) != 0ull ? 1u : 0u;
    const int w = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        s_m[w] = m;
        s_f[w] = f;
    }
    __syncthreads();
    m = s_m[0];
    f = s_f[0];
    for (int j = 1; j < PREP_THREADS / WAVE; ++j) {
        m = max(m, s_m[j]);
        f |= s_f[j];
    }
    __syncthreads();
}

// 1. dose maximum and finiteness of D_r (WITH_EV: of D_e too), one partial per block (vb
// of vgrid).  The map's compaction checks D_e where it loads it (prep_count_body); there
// block 0 here clears the flags that the later kernels or into.
template <bool WITH_EV>
__device__ __forceinline__ void dose_max_body(const PrepArgs& a, int vb, int vgrid) {
    uint32_t best = 0u, bad = 0u;
    // DM_ITEMS nodes per thread per step, all loads of a step issued before the first use
    // (indices clamped to the last node; the clamped copies do not change a max or an or)
    constexpr int DM_ITEMS = 8;
    const int64_t step = (int64_t)vgrid * PREP_THREADS * DM_ITEMS;
    for (int64_t b0 = (int64_t)vb * PREP_THREADS * DM_ITEMS; b0 < a.n; b0 += step) {
        float r[DM_ITEMS], e[DM_ITEMS];
#pragma unroll
        for (int k = 0; k < DM_ITEMS; ++k) {
            const int64_t i = b0 + (int64_t)k * PREP_THREADS + threadIdx.x;
            const int64_t j = i < a.n ? i : a.n - 1;
            r[k] = a.ref[j];
            if (WITH_EV) e[k] = a.ev[j];
        }
#pragma unroll
        for (int k = 0; k < DM_ITEMS; ++k) {
            bad |= (!isfinite(r[k]) || (WITH_EV && !isfinite(e[k]))) ? 1u : 0u;
            best = max(best, float_to_ord(r[k]));
        }
    }
    block_max_or(best, bad);
    if (threadIdx.x == 0) {
        a.part[vb] = best;
        a.part[MAX_BLOCKS + vb] = bad;
        if (!WITH_EV && vb == 0) a.sc->flags = 0u;
    }
    if (a.super && vb == 0)
        for (int j = threadIdx.x; j < 2 * a.n_super; j += PREP_THREADS) a.super[j] = 0u;
}

__global__ __launch_bounds__(PREP_THREADS) void k_dose_max(PrepArgs a) {
    dose_max_body<false>(a, blockIdx.x, gridDim.x);
}
__global__ __launch_bounds__(PREP_THREADS) void k_dose_max_both(PrepArgs a) {
    dose_max_body<true>(a, blockIdx.x, gridDim.x);
}

// 1b. dose maximum and the global 1/dD only (no mask, no compaction): one block reduces
// the partials of k_dose_max.
__global__ __launch_bounds__(PREP_THREADS) void k_dose_finish(PrepArgs a, int nb_red) {
    uint32_t dm = 0u, bad = 0u;
    for (int j = threadIdx.x; j < nb_red; j += PREP_THREADS) {
        dm = max(dm, a.part[j]);
        bad |= a.part[MAX_BLOCKS + j];
    }
    block_max_or(dm, bad);
    if (threadIdx.x == 0) {
        const float dmax = ord_to_float(dm);
        a.sc->dmax_ord = dm;
        a.sc->flags = bad ? FLAG_NONFINITE : 0u;
        a.sc->thr_val = a.thr * dmax;
        a.sc->inv_dd = 1.0f / (a.dd * dmax);
    }
}

__device__ __forceinline__ bool node_masked(float dr, float thr_val, int local) {
    return dr >= thr_val && (!local || dr > 0.0f);
}

// 2. every block: the dose maximum from the partials, then per tile the masked count, max
// gamma0^2 and -1 for unmasked nodes.  Block 0 stores the scalars of this map.
__device__ __forceinline__ void prep_count_body(const PrepArgs& a, int nb_red, int vb) {
    // this tile's doses first (they do not depend on the dose maximum), then the partials:
    // all loads in flight together, indices clamped to valid entries
    const int64_t base = (int64_t)vb * PREP_TILE;
    float rr[PREP_ITEMS], ee[PREP_ITEMS];
#pragma unroll
    for (int k = 0; k < PREP_ITEMS; ++k) {
        const int64_t i = base + (int64_t)k * PREP_THREADS + threadIdx.x;
        const int64_t j = i < a.n ? i : a.n - 1;
        rr[k] = a.ref[j];
        ee[k] = a.ev[j];
    }
    constexpr int PR = MAX_BLOCKS / PREP_THREADS;
    uint32_t pm[PR], pb[PR];
#pragma unroll
    for (int r = 0; r < PR; ++r) {
        const int j = threadIdx.x + PREP_THREADS * r;
        const int jj = j < nb_red ? j : 0;
        pm[r] = a.part[jj];
        pb[r] = a.part[MAX_BLOCKS + jj];
    }
    uint32_t dm = 0u, bad = 0u;
#pragma unroll
    for (int r = 0; r < PR; ++r) {
        dm = max(dm, pm[r]);
        bad |= pb[r];
    }
    block_max_or(dm, bad);
    const float dmax = ord_to_float(dm);
    const float thr_val = a.thr * dmax;
    const float inv_dd_g = 1.0f / (a.dd * dmax);
    if (vb == 0) {
        for (int j = threadIdx.x; j < SUM_BINS; j += PREP_THREADS) a.sums[j] = BlockSums{};
        if (threadIdx.x == 0) {
            Scalars* sc = a.sc;
            sc->dmax_ord = dm;
            if (bad) atomicOr(&sc->flags, FLAG_NONFINITE);
            sc->thr_val = thr_val;
            sc->inv_dd = inv_dd_g;
            sc->r2_bits = 0u;
            sc->n_masked = 0u;
            sc->n_tail = 0u;
            sc->n_guard = 0u;
            sc->maxg2_bits = 0u;
            sc->n_fallback = 0u;
            sc->sort_overflow = 0u;
            sc->long_rows = 0u;
            sc->n_fallback_inline = 0u;
            sc->n_pass = 0ull;
            sc->n_border = 0ull;
            sc->n_fp64 = 0ull;
            sc->n_cells = 0ull;
        }
    }
    uint32_t cnt = 0u, best = 0u;
    bool bad_e = false;
    const int lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int k = 0; k < PREP_ITEMS; ++k) {
        const int64_t i = base + (int64_t)k * PREP_THREADS + threadIdx.x;
        bool m = false;
        if (i < a.n) {
            const float dr = rr[k];
            bad_e |= !isfinite(ee[k]);
            m = node_masked(dr, thr_val, a.local);
            if (m) {
                const float de = ee[k];
                const float g2 = gamma0_sq(de, dr, node_inv_dd(dr, inv_dd_g, a.dd, a.local));
                best = max(best, f2u(g2));
                ++cnt;
            } else {
                a.gamma[i] = -1.0f;
            }
        }
        // the mask bits of the wave's 64 consecutive nodes, for the emit
        const unsigned long long bal = __ballot(m);
        if (lane == 0) a.mbits[(base + (int64_t)k * PREP_THREADS + (threadIdx.x & ~(WAVE - 1))) / WAVE] = bal;
    }
    if (__ballot(bad_e) != 0ull && lane == 0) atomicOr(&a.sc->flags, FLAG_NONFINITE);
    __shared__ uint32_t s_cnt[PREP_THREADS / WAVE];
    cnt = wave_sum_u32(cnt);
    if ((threadIdx.x & (WAVE - 1)) == 0) s_cnt[threadIdx.x / WAVE] = cnt;
    uint32_t unused = 0u;
    block_max_or(best, unused);   // also orders s_cnt
    if (threadIdx.x == 0) {
        uint32_t c = 0u;
        for (int j = 0; j < PREP_THREADS / WAVE; ++j) c += s_cnt[j];
        a.blockcnt[vb] = c;
        const int grp = vb >> a.super_shift;
        if (c) atomicAdd(&a.super[grp], c);
        if (best) atomicMax(&a.super[a.n_super + grp], best);
    }
}

__global__ __launch_bounds__(PREP_THREADS) void k_prep_count(PrepArgs a, int nb_red) {
    prep_count_body(a, nb_red, blockIdx.x);
}

// 3. the masked nodes in grid order.
__device__ __forceinline__ void prep_emit_body(const PrepArgs& a, int vb) {
    const int64_t base = (int64_t)vb * PREP_TILE;
    __shared__ uint32_t s_wave[PREP_ITEMS][PREP_THREADS / WAVE];
    __shared__ uint32_t s_pre[PREP_THREADS / WAVE];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    // this tile's mask bits (one word per wave and item), in flight while the prefix is summed
    unsigned long long bal[PREP_ITEMS];
#pragma unroll
    for (int k = 0; k < PREP_ITEMS; ++k) bal[k] = a.mbits[(base + (int64_t)k * PREP_THREADS) / WAVE + w];
    // first slot of this tile: the groups before its own, then its group's earlier tiles
    {
        const int grp = vb >> a.super_shift;
        uint32_t v = 0u;
        for (int j = threadIdx.x; j < grp; j += PREP_THREADS) v += a.super[j];
        for (int t = (grp << a.super_shift) + threadIdx.x; t < vb; t += PREP_THREADS) v += a.blockcnt[t];
        v = wave_sum_u32(v);
        if (lane == 0) s_pre[w] = v;
    }
    bool m[PREP_ITEMS];
#pragma unroll
    for (int k = 0; k < PREP_ITEMS; ++k) {
        m[k] = (bal[k] >> lane) & 1ull;
        if (lane == 0) s_wave[k][w] = (uint32_t)__popcll(bal[k]);
    }
    __syncthreads();
    uint32_t run = 0u;
    for (int j = 0; j < PREP_THREADS / WAVE; ++j) run += s_pre[j];
#pragma unroll
    for (int k = 0; k < PREP_ITEMS; ++k) {
        uint32_t off = run, tot = 0u;
        for (int j = 0; j < PREP_THREADS / WAVE; ++j) {
            const uint32_t c = s_wave[k][j];
            if (j < w) off += c;
            tot += c;
        }
        if (m[k]) a.nodes[off + (uint32_t)__popcll(bal[k] & lt)] = (uint32_t)(base + (int64_t)k * PREP_THREADS + threadIdx.x);
        run += tot;
    }
    if (vb == a.ntiles - 1) {
        // the last tile: M and R^2 (the maximum over the groups)
        uint32_t mx = 0u, none = 0u;
        for (int j = threadIdx.x; j < a.n_super; j += PREP_THREADS) mx = max(mx, a.super[a.n_super + j]);
        block_max_or(mx, none);
        if (threadIdx.x == 0) {
            a.sc->n_masked = run;
            a.sc->r2_bits = mx;
        }
    }
}

__global__ __launch_bounds__(PREP_THREADS) void k_prep_emit(PrepArgs a) { prep_emit_body(a, blockIdx.x); }

__global__ __launch_bounds__(256) void k_pass_count(const float* __restrict__ g, int64_t n,
                                                    unsigned long long* counts) {
    uint32_t ne = 0u, np = 0u, nb = 0u;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float v = g[i];
        ne += v >= 0.0f;
        np += (v >= 0.0f) & (v <= 1.0f);
        nb += (v >= 0.0f) & (fabsf(v - 1.0f) <= 1e-5f);
    }
    // summed over the block, then one atomic per count (one per wave on these three
    // addresses serialises)
    __shared__ uint32_t s[3][256 / WAVE];
    ne = wave_sum_u32(ne);
    np = wave_sum_u32(np);
    nb = wave_sum_u32(nb);
    const int w = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        s[0][w] = ne;
        s[1][w] = np;
        s[2][w] = nb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t[3] = {0ull, 0ull, 0ull};
        for (int j = 0; j < (int)(blockDim.x / WAVE); ++j)
            for (int q = 0; q < 3; ++q) t[q] += s[q][j];
        for (int q = 0; q < 3; ++q)
            if (t[q]) atomicAdd(&counts[q], t[q]);
    }
}

__global__ void k_zero3(unsigned long long* c) {
    if (threadIdx.x < 3) c[threadIdx.x] = 0ull;
}

int reduce_blocks(int64_t n) {
    int64_t b = (n + PREP_THREADS * 8 - 1) / (PREP_THREADS * 8);
    if (b > MAX_BLOCKS) b = MAX_BLOCKS;
    return (int)(b < 1 ? 1 : b);
}

// Batches: the same bodies, one block per (pair, block) item.
__global__ __launch_bounds__(PREP_THREADS) void k_batch_dose_max(const BatchPair* __restrict__ pairs,
                                                                 const uint2* __restrict__ items) {
    const uint2 w = items[blockIdx.x];
    const BatchPair& P = pairs[w.x];
    dose_max_body<false>(P.pa, (int)w.y, P.nbr);
}
__global__ __launch_bounds__(PREP_THREADS) void k_batch_prep_count(const BatchPair* __restrict__ pairs,
                                                                   const uint2* __restrict__ items) {
    const uint2 w = items[blockIdx.x];
    const BatchPair& P = pairs[w.x];
    prep_count_body(P.pa, P.nbr, (int)w.y);
}
__global__ __launch_bounds__(PREP_THREADS) void k_batch_prep_emit(const BatchPair* __restrict__ pairs,
                                                                  const uint2* __restrict__ items) {
    const uint2 w = items[blockIdx.x];
    const BatchPair& P = pairs[w.x];
    prep_emit_body(P.pa, (int)w.y);
}

}  // namespace

int prep_reduce_blocks(int64_t n) { return reduce_blocks(n); }

hipError_t launch_batch_prep(const BatchPair* pairs, const uint2* dm, int n_dm, const uint2* tiles, int n_tiles,
                             hipStream_t s) {
    if (n_dm <= 0 || n_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_dose_max, dim3((unsigned)n_dm), dim3(PREP_THREADS), 0, s, pairs, dm);
    hipLaunchKernelGGL(k_batch_prep_count, dim3((unsigned)n_tiles), dim3(PREP_THREADS), 0, s, pairs, tiles);
    hipLaunchKernelGGL(k_batch_prep_emit, dim3((unsigned)n_tiles), dim3(PREP_THREADS), 0, s, pairs, tiles);
    return hipGetLastError();
}

int64_t prep_tiles(int64_t n) { return (n + PREP_TILE - 1) / PREP_TILE; }

void prep_groups(int64_t n, int* shift, int* n_super) {
    // 2^sh tiles per group with 4^(sh + 3) >= tiles: about sqrt(tiles) / 8 tiles share a
    // group counter (same-address atomics from blocks on every XCD serialise), and the
    // emit reads about 8 sqrt(tiles) group sums
    const int64_t t = prep_tiles(n);
    int sh = 0;
    while (((int64_t)1 << (2 * (sh + 3))) < t) ++sh;
    *shift = sh;
    *n_super = (int)((t + ((int64_t)1 << sh) - 1) >> sh);
}

int64_t prep_mbits_offset(int64_t n) {
    int sh = 0, ns = 0;
    prep_groups(n, &sh, &ns);
    return (prep_tiles(n) + 2 * (int64_t)ns + 1) & ~(int64_t)1;   // 8-byte aligned
}

int64_t prep_words(int64_t n) { return prep_mbits_offset(n) + 2 * prep_tiles(n) * (PREP_TILE / 64); }

hipError_t launch_prep(const PrepArgs& a, hipStream_t s) {
    const int nbr = reduce_blocks(a.n);
    const int64_t nb = prep_tiles(a.n);
    hipLaunchKernelGGL(k_dose_max, dim3(nbr), dim3(PREP_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_prep_count, dim3((unsigned)nb), dim3(PREP_THREADS), 0, s, a, nbr);
    hipLaunchKernelGGL(k_prep_emit, dim3((unsigned)nb), dim3(PREP_THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_dose_scalars(const PrepArgs& a, hipStream_t s) {
    const int nbr = reduce_blocks(a.n);
    hipLaunchKernelGGL(k_dose_max_both, dim3(nbr), dim3(PREP_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_dose_finish, dim3(1), dim3(PREP_THREADS), 0, s, a, nbr);
    return hipGetLastError();
}

hipError_t launch_pass_count(const float* gamma, int64_t n, unsigned long long* counts3, hipStream_t s) {
    int64_t b = (n + 255) / 256;
    if (b > MAX_BLOCKS) b = MAX_BLOCKS;
    if (b < 1) b = 1;
    hipLaunchKernelGGL(k_zero3, dim3(1), dim3(64), 0, s, counts3);
    hipLaunchKernelGGL(k_pass_count, dim3((unsigned)b), dim3(256), 0, s, gamma, n, counts3);
    return hipGetLastError();
}

}  // namespace gammax
