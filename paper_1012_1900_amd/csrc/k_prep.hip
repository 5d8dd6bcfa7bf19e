// Normalisation, mask, gamma0 and ordered compaction (Algorithm A2 step 2, "Kernel 1"),
// plus the stand-alone pass-rate reduction.  Every pass streams the dose arrays with
// coalesced loads; reductions go through per-block partials and one finishing block, so
// no address is hit by thousands of atomics.
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

// Block-wide max and or over 256 threads (result valid in thread 0).
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
    if (threadIdx.x == 0) {
        for (int j = 1; j < PREP_THREADS / WAVE; ++j) {
            m = max(m, s_m[j]);
            f |= s_f[j];
        }
    }
}

// max D_r and a finiteness check of both doses: grid-stride, one partial per block.
__global__ __launch_bounds__(PREP_THREADS) void k_dose_max(const float* __restrict__ ref,
                                                           const float* __restrict__ ev, int64_t n,
                                                           uint32_t* __restrict__ part) {
    uint32_t best = 0u, bad = 0u;
    const int64_t stride = (int64_t)gridDim.x * PREP_THREADS;
    for (int64_t i = (int64_t)blockIdx.x * PREP_THREADS + threadIdx.x; i < n; i += stride) {
        const float r = ref[i];
        const float e = ev[i];
        bad |= (!isfinite(r) || !isfinite(e)) ? 1u : 0u;
        best = max(best, float_to_ord(r));
    }
    block_max_or(best, bad);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = best;
        part[MAX_BLOCKS + blockIdx.x] = bad;
    }
}

// One block: reduce the partials, set the threshold and global 1/dD, clear the counters.
__global__ __launch_bounds__(PREP_THREADS) void k_finish_max(const uint32_t* __restrict__ part, int nb,
                                                             Scalars* sc, float thr, float dd,
                                                             BlockSums* sums) {
    for (int j = threadIdx.x; j < SUM_BINS; j += PREP_THREADS) sums[j] = BlockSums{};
    uint32_t m = 0u, f = 0u;
    for (int j = threadIdx.x; j < nb; j += PREP_THREADS) {
        m = max(m, part[j]);
        f |= part[MAX_BLOCKS + j];
    }
    block_max_or(m, f);
    if (threadIdx.x == 0) {
        const float dmax = ord_to_float(m);
        sc->dmax_ord = m;
        sc->flags = f ? FLAG_NONFINITE : 0u;
        sc->thr_val = thr * dmax;
        sc->inv_dd = 1.0f / (dd * dmax);
        sc->r2_bits = 0u;
        sc->n_masked = 0u;
        sc->n_tail = 0u;
        sc->n_guard = 0u;
        sc->maxg2_bits = 0u;
        sc->n_pass = 0ull;
        sc->n_border = 0ull;
        sc->n_fp64 = 0ull;
        sc->n_cells = 0ull;
    }
}

__device__ __forceinline__ bool node_masked(float dr, float thr_val, int local) {
    return dr >= thr_val && (!local || dr > 0.0f);
}

// Pass 1: per tile, count masked nodes, take max gamma0^2, write -1 for unmasked nodes.
__global__ __launch_bounds__(PREP_THREADS) void k_prep_count(PrepArgs a) {
    const float thr_val = a.sc->thr_val;
    const float inv_dd_g = a.sc->inv_dd;
    const int64_t base = (int64_t)blockIdx.x * PREP_TILE;
    uint32_t cnt = 0u, best = 0u;
#pragma unroll 4
    for (int k = 0; k < PREP_ITEMS; ++k) {
        const int64_t i = base + (int64_t)k * PREP_THREADS + threadIdx.x;
        if (i < a.n) {
            const float dr = a.ref[i];
            if (node_masked(dr, thr_val, a.local)) {
                const float de = a.ev[i];
                const float g2 = gamma0_sq(de, dr, node_inv_dd(dr, inv_dd_g, a.dd, a.local));
                best = max(best, f2u(g2));
                ++cnt;
            } else {
                a.gamma[i] = -1.0f;
            }
        }
    }
    __shared__ uint32_t s_cnt[PREP_THREADS / WAVE], s_max[PREP_THREADS / WAVE];
    cnt = wave_sum_u32(cnt);
    best = wave_max_u32(best);
    const int w = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        s_cnt[w] = cnt;
        s_max[w] = best;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t c = 0u, m = 0u;
        for (int j = 0; j < PREP_THREADS / WAVE; ++j) {
            c += s_cnt[j];
            m = max(m, s_max[j]);
        }
        a.blockcnt[blockIdx.x] = c;
        a.blockmax[blockIdx.x] = m;
    }
}

// Pass 2 (one workgroup): exclusive scan of the tile counts, M and R^2 into the scalars.
__global__ __launch_bounds__(1024) void k_scan_blocks(uint32_t* cnt, const uint32_t* bmax, int64_t nb,
                                                      Scalars* sc) {
    __shared__ uint32_t s_wave[1024 / WAVE];
    __shared__ uint32_t s_wmax[1024 / WAVE];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0u;
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    uint32_t mx = 0u;
    for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
        const int64_t i = b0 + threadIdx.x;
        const uint32_t v = i < nb ? cnt[i] : 0u;
        if (i < nb) mx = max(mx, bmax[i]);
        uint32_t x = v;
        for (int o = 1; o < WAVE; o <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)x, o);
            if (lane >= o) x += y;
        }
        if (lane == WAVE - 1) s_wave[w] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t run = s_carry;
            for (int j = 0; j < 1024 / WAVE; ++j) {
                const uint32_t t = s_wave[j];
                s_wave[j] = run;
                run += t;
            }
            s_carry = run;
        }
        __syncthreads();
        if (i < nb) cnt[i] = s_wave[w] + x - v;
        __syncthreads();
    }
    mx = wave_max_u32(mx);
    if (lane == 0) s_wmax[w] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t m = 0u;
        for (int j = 0; j < 1024 / WAVE; ++j) m = max(m, s_wmax[j]);
        sc->n_masked = s_carry;
        sc->r2_bits = m;
    }
}

// Pass 3: the masked nodes in grid order.
__global__ __launch_bounds__(PREP_THREADS) void k_prep_emit(PrepArgs a) {
    const float thr_val = a.sc->thr_val;
    const int64_t base = (int64_t)blockIdx.x * PREP_TILE;
    __shared__ uint32_t s_wave[PREP_THREADS / WAVE];
    uint32_t run = a.blockcnt[blockIdx.x];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
    for (int k = 0; k < PREP_ITEMS; ++k) {
        const int64_t i = base + (int64_t)k * PREP_THREADS + threadIdx.x;
        const bool m = i < a.n && node_masked(a.ref[i], thr_val, a.local);
        const unsigned long long bal = __ballot(m);
        if (lane == 0) s_wave[w] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t off = run, tot = 0u;
        for (int j = 0; j < PREP_THREADS / WAVE; ++j) {
            const uint32_t c = s_wave[j];
            if (j < w) off += c;
            tot += c;
        }
        if (m) a.nodes[off + (uint32_t)__popcll(bal & lt)] = (uint32_t)i;
        run += tot;
        __syncthreads();
    }
}

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
    ne = wave_sum_u32(ne);
    np = wave_sum_u32(np);
    nb = wave_sum_u32(nb);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        if (ne) atomicAdd(&counts[0], (unsigned long long)ne);
        if (np) atomicAdd(&counts[1], (unsigned long long)np);
        if (nb) atomicAdd(&counts[2], (unsigned long long)nb);
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

}  // namespace

hipError_t launch_prep(const PrepArgs& a, hipStream_t s) {
    const int nbr = reduce_blocks(a.n);
    const int64_t nb = (a.n + PREP_TILE - 1) / PREP_TILE;
    hipLaunchKernelGGL(k_dose_max, dim3(nbr), dim3(PREP_THREADS), 0, s, a.ref, a.ev, a.n, a.part);
    hipLaunchKernelGGL(k_finish_max, dim3(1), dim3(PREP_THREADS), 0, s, a.part, nbr, a.sc, a.thr, a.dd, a.sums);
    hipLaunchKernelGGL(k_prep_count, dim3((unsigned)nb), dim3(PREP_THREADS), 0, s, a);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, a.blockcnt, a.blockmax, nb, a.sc);
    hipLaunchKernelGGL(k_prep_emit, dim3((unsigned)nb), dim3(PREP_THREADS), 0, s, a);
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
