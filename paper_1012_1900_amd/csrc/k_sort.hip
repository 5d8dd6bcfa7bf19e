// Stable LSD radix sort of (uint32 key, uint32 value) pairs, 4 passes of 8 bits.
//
// Used for the DD sort of the reference nodes (Algorithm A2 step 3) and for the cell
// table (step 5).  Per pass: a per-tile digit histogram (LDS atomics), a per-digit scan
// over tiles, and a stable scatter in which each wave ranks its 64 elements by digit
// with eight ballots (lanes sharing a digit form a peer mask) and the LDS holds the
// running per-digit offsets of the tile.
#include "internal.hpp"

namespace gammax {

namespace {

constexpr int WAVE = 64;
constexpr int SORT_THREADS = 256;
constexpr int SORT_CHUNKS = 4;
constexpr int SORT_TILE = SORT_THREADS * SORT_CHUNKS;
constexpr int RADIX = 256;
constexpr int NWAVES = SORT_THREADS / WAVE;

__device__ __forceinline__ int64_t count_of(int64_t n_max, const uint32_t* n_dev) {
    return n_dev ? (int64_t)*n_dev : n_max;
}

// Sort keys from a caller's per-node key (non-negative floats order as their bits).
__global__ __launch_bounds__(SORT_THREADS) void k_given_keys(const uint32_t* __restrict__ nodes,
                                                             const uint32_t* __restrict__ count,
                                                             const float* __restrict__ given,
                                                             uint32_t* __restrict__ key) {
    const uint32_t n = *count;
    for (uint32_t i = blockIdx.x * SORT_THREADS + threadIdx.x; i < n; i += gridDim.x * SORT_THREADS) {
        const float v = given[nodes[i]];
        key[i] = __float_as_uint(v > 0.0f ? v : 0.0f);   // NaN and negatives: 0
    }
}

__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                             int64_t n_max, const uint32_t* n_dev,
                                                             int shift, uint32_t* __restrict__ hist,
                                                             int64_t nb) {
    const int64_t n = count_of(n_max, n_dev);
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    if (base >= n) return;   // uniform: the scan and the scatter use only the tiles that exist
    __shared__ uint32_t h[RADIX];
    h[threadIdx.x] = 0u;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SORT_CHUNKS; ++k) {
        int64_t i = base + (int64_t)k * SORT_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (RADIX - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Block-wide exclusive scan of one value per thread; returns the exclusive prefix and
// writes the block total to *total.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_wave,
                                                         uint32_t* total) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    uint32_t x = v;
    for (int o = 1; o < WAVE; o <<= 1) {
        uint32_t y = (uint32_t)__shfl_up((int)x, o);
        if (lane >= o) x += y;
    }
    if (lane == WAVE - 1) s_wave[w] = x;
    __syncthreads();
    uint32_t off = 0u, tot = 0u;
    for (int j = 0; j < NWAVES; ++j) {
        uint32_t c = s_wave[j];
        if (j < w) off += c;
        tot += c;
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

// One workgroup per digit: exclusive scan of that digit's counts over the tiles that hold
// elements (the first ceil(n / SORT_TILE) of the nb the grid was sized for).
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scan(uint32_t* __restrict__ hist, int64_t nb,
                                                             int64_t n_max, const uint32_t* n_dev,
                                                             uint32_t* __restrict__ totals) {
    __shared__ uint32_t s_wave[NWAVES];
    const int64_t n = count_of(n_max, n_dev);
    const int64_t used = min(nb, (n + SORT_TILE - 1) / SORT_TILE);
    uint32_t* row = hist + (int64_t)blockIdx.x * nb;
    uint32_t carry = 0u;
    for (int64_t b0 = 0; b0 < used; b0 += SORT_THREADS) {
        int64_t i = b0 + threadIdx.x;
        uint32_t v = i < used ? row[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(v, s_wave, &tot);
        if (i < used) row[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, int64_t n_max, const uint32_t* n_dev, int shift,
    const uint32_t* __restrict__ hist, const uint32_t* __restrict__ totals, int64_t nb) {
    const int64_t n = count_of(n_max, n_dev);
    if ((int64_t)blockIdx.x * SORT_TILE >= n) return;   // uniform: nothing of this tile exists
    __shared__ uint32_t s_base[RADIX];
    __shared__ uint32_t s_wcnt[NWAVES][RADIX];
    __shared__ uint32_t s_wave[NWAVES];
    const int t = threadIdx.x;
    {
        uint32_t tot;
        uint32_t ex = block_exclusive_scan(totals[t], s_wave, &tot);
        s_base[t] = ex + hist[(int64_t)t * nb + blockIdx.x];
        for (int w = 0; w < NWAVES; ++w) s_wcnt[w][t] = 0u;
    }
    __syncthreads();
    const int lane = t & (WAVE - 1), w = t / WAVE;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    // every chunk's pair is loaded before the first is ranked: one memory latency per tile
    uint32_t keys[SORT_CHUNKS], vals[SORT_CHUNKS];
#pragma unroll
    for (int k = 0; k < SORT_CHUNKS; ++k) {
        const int64_t i = base + (int64_t)k * SORT_THREADS + t;
        const int64_t j = i < n ? i : n - 1;   // n > base: the clamped index is in range
        keys[k] = kin[j];
        vals[k] = vin[j];
    }
#pragma unroll
    for (int k = 0; k < SORT_CHUNKS; ++k) {
        const int64_t i = base + (int64_t)k * SORT_THREADS + t;
        const bool valid = i < n;
        const uint32_t key = valid ? keys[k] : 0u, val = vals[k];
        const uint32_t dig = (key >> shift) & (RADIX - 1);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0u) s_wcnt[w][dig] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = s_base[dig] + rank;
            for (int j = 0; j < w; ++j) pos += s_wcnt[j][dig];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0u;
        for (int j = 0; j < NWAVES; ++j) {
            add += s_wcnt[j][t];
            s_wcnt[j][t] = 0u;
        }
        s_base[t] += add;
        __syncthreads();
    }
}

// Short lists: each element's place is the number of smaller keys plus the number of
// equal keys before it (a stable rank), i.e. the number of smaller (key, position) pairs.
// A workgroup of 16 waves ranks 64 keys: it holds the whole list in LDS as 64-bit
// (key << 32 | position) words, distinct and ordered as the stable order, and each wave
// counts the words below its 64 against one sixteenth of the list (broadcast reads, one
// 64-bit compare and one add per word), the sixteen counts then summed in LDS.  For
// n <= SMALL_SORT_CAP; a longer list is left as it is and *overflow set (the callers sort
// only to order work, so any order is correct).
// ORDER_ONLY: the values are the positions 0..n-1 (a work list in its queue order); the
// sorted positions are written straight into `vals` and the keys are not moved.
// Otherwise the pairs go to the scratch arrays at their places and a second pass copies
// them back.
constexpr int SMALL_THREADS = 1024;
constexpr int SMALL_KEYS = 64;    // keys ranked per workgroup
constexpr int SMALL_PARTS = SMALL_THREADS / SMALL_KEYS;
constexpr int SMALL_BLOCKS = SMALL_SORT_CAP / SMALL_KEYS;
static_assert(SMALL_SORT_CAP % SMALL_THREADS == 0 && SMALL_KEYS % (4 * SMALL_PARTS) == 0,
              "each part of the padded list must be a whole number of 4-word steps");
template <bool ORDER_ONLY>
__global__ __launch_bounds__(SMALL_THREADS) void k_sort_small_rank(const uint32_t* __restrict__ keys,
                                                                   uint32_t* __restrict__ vals,
                                                                   uint32_t* __restrict__ tk, uint32_t* __restrict__ tv,
                                                                   const uint32_t* n_dev, uint32_t* overflow) {
    __shared__ __align__(16) uint64_t sk[SMALL_SORT_CAP];
    __shared__ uint32_t s_part[SMALL_PARTS][SMALL_KEYS];
    const uint32_t n = *n_dev;
    if (n > (uint32_t)SMALL_SORT_CAP) {
        if (blockIdx.x == 0 && threadIdx.x == 0) *overflow = 1u;
        return;
    }
    if (blockIdx.x * SMALL_KEYS >= n) return;
    // the list padded to a multiple of 64 with all-ones words (above every real word);
    // every thread issues all its loads (clamped to the last key) before the first store,
    // so the staging costs one memory latency
    const uint32_t n64 = (n + 63u) & ~63u;
    {
        constexpr int R = SMALL_SORT_CAP / SMALL_THREADS;
        uint32_t v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint32_t j = threadIdx.x + SMALL_THREADS * r;
            v[r] = keys[j < n ? j : n - 1];
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            asm volatile("" : "+v"(v[r]));
            const uint32_t j = threadIdx.x + SMALL_THREADS * r;
            if (j < n64) sk[j] = j < n ? ((uint64_t)v[r] << 32 | j) : ~0ull;
        }
    }
    __syncthreads();
    const uint32_t lane = threadIdx.x & (SMALL_KEYS - 1), part = threadIdx.x / SMALL_KEYS;
    const uint32_t i = blockIdx.x * SMALL_KEYS + lane;
    const uint64_t k = sk[i < n ? i : 0];
    // this wave's part [j0, j1) of the padded list (a multiple of 4 long)
    const uint32_t q = n64 / SMALL_PARTS;
    const uint32_t j0 = part * q, j1 = j0 + q;
    uint32_t cnt = 0;
    const ulonglong2* s2 = reinterpret_cast<const ulonglong2*>(sk);
    for (uint32_t j = j0; j < j1; j += 4) {
        const ulonglong2 a = s2[j >> 1], b = s2[(j >> 1) + 1];
        cnt += (a.x < k ? 1u : 0u) + (a.y < k ? 1u : 0u) + (b.x < k ? 1u : 0u) + (b.y < k ? 1u : 0u);
    }
    s_part[part][lane] = cnt;
    __syncthreads();
    if (part != 0 || i >= n) return;
    uint32_t rank = 0;
#pragma unroll
    for (int p = 0; p < SMALL_PARTS; ++p) rank += s_part[p][lane];
    if (ORDER_ONLY) {
        vals[rank] = i;
    } else {
        tk[rank] = (uint32_t)(k >> 32);
        tv[rank] = vals[i];
    }
}

__global__ __launch_bounds__(SMALL_THREADS) void k_sort_small_copy(uint32_t* __restrict__ keys,
                                                                   uint32_t* __restrict__ vals,
                                                                   const uint32_t* __restrict__ tk,
                                                                   const uint32_t* __restrict__ tv,
                                                                   const uint32_t* n_dev) {
    const uint32_t n = *n_dev;
    if (n > (uint32_t)SMALL_SORT_CAP) return;
    for (uint32_t i = blockIdx.x * SMALL_THREADS + threadIdx.x; i < n; i += gridDim.x * SMALL_THREADS) {
        keys[i] = tk[i];
        vals[i] = tv[i];
    }
}

}  // namespace

hipError_t sort_pairs_small(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals,
                            const uint32_t* n_dev, uint32_t* overflow, hipStream_t s) {
    hipLaunchKernelGGL(k_sort_small_rank<false>, dim3(SMALL_BLOCKS), dim3(SMALL_THREADS), 0, s, keys, vals,
                       tmp_keys, tmp_vals, n_dev, overflow);
    hipLaunchKernelGGL(k_sort_small_copy, dim3(SMALL_SORT_CAP / SMALL_THREADS), dim3(SMALL_THREADS), 0, s, keys,
                       vals, tmp_keys, tmp_vals, n_dev);
    return hipGetLastError();
}

hipError_t sort_order_small(const uint32_t* keys, uint32_t* order, const uint32_t* n_dev, uint32_t* overflow,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_sort_small_rank<true>, dim3(SMALL_BLOCKS), dim3(SMALL_THREADS), 0, s, keys, order,
                       nullptr, nullptr, n_dev, overflow);
    return hipGetLastError();
}

int64_t sort_hist_words(int64_t n_max) {
    const int64_t nb = (n_max + SORT_TILE - 1) / SORT_TILE;
    return (int64_t)RADIX * (nb > 0 ? nb : 1) + RADIX;
}

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* tmp_keys, uint32_t* tmp_vals,
                            int64_t n_max, const uint32_t* n_dev, uint32_t* hist, hipStream_t s, int low_bit) {
    if (n_max <= 1) return hipSuccess;
    if (low_bit < 0 || low_bit > 24 || low_bit % 16 != 0) return hipErrorInvalidValue;   // an even pass count
    const int64_t nb = (n_max + SORT_TILE - 1) / SORT_TILE;
    uint32_t* totals = hist + (int64_t)RADIX * nb;
    uint32_t *ki = keys, *vi = vals, *ko = tmp_keys, *vo = tmp_vals;
    for (int shift = low_bit; shift < 32; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(SORT_THREADS), 0, s, ki, n_max, n_dev,
                           shift, hist, nb);
        hipLaunchKernelGGL(k_radix_scan, dim3(RADIX), dim3(SORT_THREADS), 0, s, hist, nb, n_max, n_dev, totals);
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(SORT_THREADS), 0, s, ki, vi, ko, vo,
                           n_max, n_dev, shift, hist, totals, nb);
        uint32_t* tk = ki;
        ki = ko;
        ko = tk;
        uint32_t* tv = vi;
        vi = vo;
        vo = tv;
    }
    return hipGetLastError();
}

hipError_t launch_given_keys(const uint32_t* nodes, const uint32_t* count, const float* given, uint32_t* key,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_given_keys, dim3(512), dim3(SORT_THREADS), 0, s, nodes, count, given, key);
    return hipGetLastError();
}

}  // namespace gammax
