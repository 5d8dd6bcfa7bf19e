// The learned search radius: a 3D CNN that predicts log(gamma + 0.01) at every node from
// the 9x9x9 neighbourhood of two dose features, with its training kernels.  Not part of
// the paper's method; an addition around it (its output only orders and bounds the
// search, never changes a gamma value).
//
// Network: four valid 3x3x3 convolutions, channels 2 -> 16 -> 16 -> 16 -> 1, ReLU after
// the first three, on features zero-padded by 4 nodes, so the output covers the grid.
// Arithmetic: bf16 operands (weights and activations, round to nearest even) on the
// matrix cores (v_mfma_f32_16x16x32_bf16), FP32 accumulation, FP32 biases; hidden
// activations are stored as bf16 after the ReLU, the last layer's output as FP32.
//
// Layouts.  Activations are channel-last: [volume][z][y][x][C] bf16 (C = 16, or 2 for the
// features), so one node's 16 channels are one 32-byte load.  A convolution is an
// implicit GEMM per 16-node row segment along x: D[co][node] = sum_k W[co][k] X[k][node],
// k = (tap, ci), in 32-wide chunks (chunk_tap gives the taps of each chunk of a 16-channel
// layer).  The weights are the A operand, packed once per update into the lane order of
// the instruction ("fragments", 16 bytes per lane per chunk); the input tile (with its
// halo) is staged in LDS and read as the B operand; each lane's result is 4 consecutive
// output channels of one node (an 8-byte store).  Inference fuses layers 1 and 2
// (k_conv12) and computes the single-channel last layer by shifts (k_conv_last); the
// network at listed nodes only runs per node from its 9^3 patch (k_cnn_tail).
//
// Backward: bwd-data is the same kernel run on the output gradient with the flipped,
// transposed kernel and an input offset of -2 (full correlation), times the ReLU mask of
// the stored activation; bwd-weight contracts over nodes (D[co][ci] per tap, both
// operands staged planar in LDS), one partial per workgroup, reduced deterministically.
#include <type_traits>

#include "internal.hpp"
#include "cnn.hpp"

namespace gammax {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct alignas(16) U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint32_t h) { return __builtin_bit_cast(float, (h & 0xFFFFu) << 16); }

// Two floats rounded to bf16 (nearest even, as f2bf for every non-NaN value) in one
// hardware conversion; `lo` in the low half.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack2bf(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}

// floor(v / E) for 0 <= v < 4096 as a multiply and a shift: with M = ceil(2^16 / E) the
// excess v (M E - 2^16) / (E 2^16) stays below 1/E there.
template <int E>
constexpr uint32_t div_magic() { return (65536u + E - 1) / E; }
template <int E>
constexpr bool div_magic_exact() {
    for (uint32_t v = 0; v < 4096; ++v)
        if (((v * div_magic<E>()) >> 16) != v / E) return false;
    return true;
}
template <int E>
__device__ __forceinline__ uint32_t div_small(uint32_t v) {
    static_assert(div_magic_exact<E>(), "multiply-shift division inexact");
    return (v * div_magic<E>()) >> 16;
}

__device__ __forceinline__ f32x4 mfma_bf16(const U4& a, const U4& b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

// Tile of workgroup b.  Workgroups are dealt to the 8 XCDs in turn (b on XCD b % 8), each
// with its own L2; neighbouring tiles share halo nodes, so XCD k takes the k-th contiguous
// eighth of the tiles (in x, then y, z order) and the halos mostly hit its L2.  A bijection
// of [0, n) whatever the dispatch order, so only locality depends on it.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int x = b & 7, k = b >> 3, q = n >> 3, r = n & 7;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

constexpr int TX = CNN_TILE_X, TY = CNN_TILE_Y, TZ = CNN_TILE_Z;
constexpr int LX = TX + 2, LY = TY + 2, LZ = TZ + 2;
constexpr int NTHREADS = 256;

__device__ __forceinline__ void tap_xyz(int t, int& dz, int& dy, int& dx) {
    dz = t / 9;
    dy = (t / 3) % 3;
    dx = t % 3;
}

// The 14 k chunks of a layer with 16 input channels: chunk c holds tap chunk_tap(c, 0) in
// k 0..15 (lane groups 0, 1 of the B operand) and tap chunk_tap(c, 1) in k 16..31 (groups
// 2, 3), 16 channels each; tap t = 9 dz + 3 dy + dx, 27 = none (zero weights).
//   c = 3 dz + dy (0..8): (dz, dy, 0) and (dz, dy, 1), an x pair;
//   c = 9 + dy:           (0, dy, 2) and (1, dy, 2);
//   c = 12:               (2, 0, 2) and (2, 1, 2);
//   c = 13:               (2, 2, 2) alone.
// The x pairs let one B operand (16 nodes of an input row, two x shifts) serve every output
// row that reads that input row, with the chunk of its (dz, dy).
__host__ __device__ constexpr int chunk_tap(int c, int h) {
    return c < 9 ? 9 * (c / 3) + 3 * (c % 3) + h
                 : (c < 12 ? 9 * h + 3 * (c - 9) + 2 : (c == 12 ? 20 + 3 * h : (h == 0 ? 26 : 27)));
}

// The k order of layer 1 (2 input channels).  Its 27 taps x 2 channels fill the 32 k slots
// of two chunks: lane group g of chunk c holds taps l1_tap(c, g, q), q = 0..3, both channels
// of each (k = 32 c + 8 g + 2 q + ci), 27 = an empty slot (zero weights).  The order was
// found by a search over the staged boxes of the dense kernels (18 x 18 x 6 and 16 x 16 x 4
// outputs) and the tail kernel (7^3) such that the four lane groups' 4-byte operand reads
// fall in distinct LDS banks (about 1.0-1.1 accesses per bank, against 1.75 for taps in
// order); every order gives the same products.
__host__ __device__ constexpr int l1_tap(int c, int g, int q) {
    constexpr int T[2][4][4] = {{{18, 26, 1, 23}, {27, 24, 0, 27}, {20, 27, 13, 21}, {19, 25, 14, 22}},
                                {{11, 17, 5, 8}, {12, 27, 4, 27}, {16, 9, 3, 6}, {15, 10, 2, 7}}};
    return T[c][g][q];
}
// The tap whose operand an empty slot reads (times a zero weight): group 0's in that slot.
__host__ __device__ constexpr int l1_read_tap(int c, int g, int q) {
    return l1_tap(c, g, q) < 27 ? l1_tap(c, g, q) : l1_tap(c, 0, q);
}
constexpr bool l1_order_valid() {
    int seen[28] = {};
    for (int c = 0; c < 2; ++c)
        for (int g = 0; g < 4; ++g)
            for (int q = 0; q < 4; ++q) ++seen[l1_tap(c, g, q)];
    for (int t = 0; t < 27; ++t)
        if (seen[t] != 1) return false;
    for (int c = 0; c < 2; ++c)
        for (int q = 0; q < 4; ++q)
            if (l1_tap(c, 0, q) >= 27) return false;
    return seen[27] == 5;
}
static_assert(l1_order_valid(), "layer 1's k order must hold every tap once, group 0 no empty slot");

// ---- forward / bwd-data convolution ----------------------------------------------------
//
// MODE 0: out = bf16(relu(acc + bias)), 16 channels.
// MODE 2: out = bf16(mask > 0 ? acc : 0), 16 channels, no bias (bwd-data with the ReLU
//         derivative of the stored activation `mask`, which has the output's shape).
// The last layer (one FP32 output channel, no ReLU) has a kernel of its own, k_conv_last.
//
// Tile: FX x FY x FZ output nodes per workgroup of 8 waves, the input tile (halo 2) and
// the weight fragments staged in LDS (76.5 KB with 16 input channels: two workgroups, 16
// waves, per compute unit).  Wave w computes the rows y0 + 2w and y0 + 2w + 1 for all FZ
// planes in one pass: 8 rows whose LDS addresses differ by immediates, so one per-lane
// address serves them all, and 8 accumulation chains alternate on the matrix core, each
// chunk's weight fragment (one LDS read) feeding 8 products.  Every row still sums its
// chunks in order 0, 1, ..., so a row's value does not depend on the grouping.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int FX = 16, FY = 16, FZ = 4;
constexpr int FLX = FX + 2, FLY = FY + 2, FLZ = FZ + 2;
constexpr int FTHREADS = 512;
constexpr int FNRY = FY / (FTHREADS / 64);   // y rows per wave
static_assert(FNRY * (FTHREADS / 64) == FY, "the waves must cover the tile's rows");

// Offset in nodes of tap t = 9 dz + 3 dy + dx within a staged forward tile.
__host__ __device__ constexpr int ftap_offset(int t) { return ((t / 9) * FLY + (t / 3) % 3) * FLX + t % 3; }

// Stage the box of BX x BY x BZ nodes with corner (gx0, gy0, gz0) of a channel-last volume
// (iz, iy, ix, CIN channels) into LDS, node-major with CIN channels per node; nodes outside
// the volume read as 0.  Thread t owns one 16-byte (16 channels) or 4-byte (2 channels) slot
// e = t % E of a box row of E slots and the rows t / E + RPR k, so its x coordinate and x
// bounds test are fixed.  All loads of a thread are issued before the first store, so the
// rounds share one memory latency (an outside node loads node 0 and stores 0).
template <int CIN, int BX, int BY, int BZ>
__device__ __forceinline__ void stage_box(const uint16_t* __restrict__ in, int ix, int iy, int iz, int gx0, int gy0,
                                          int gz0, uint16_t* tile) {
    constexpr int PER_NODE = CIN == 16 ? 2 : 1;
    constexpr int E = BX * PER_NODE, RPR = FTHREADS / E, NROW = BZ * BY;
    constexpr int ROUNDS = (NROW + RPR - 1) / RPR;
    constexpr int SLOT = CIN == 16 ? 8 : 2;   // bf16 per slot
    static_assert(ROUNDS <= 32, "one mask bit per round");
    using V = typename std::conditional<CIN == 16, u32x4, uint32_t>::type;
    const int e = threadIdx.x % E, r0 = threadIdx.x / E;
    const int gx = gx0 + e / PER_NODE;
    const bool okx = r0 < RPR && (unsigned)gx < (unsigned)ix;
    const uint16_t* pe = in + (e % PER_NODE) * 8;
    V q[ROUNDS];
    uint32_t okm = 0u;
#pragma unroll
    for (int k = 0; k < ROUNDS; ++k) {
        const int row = r0 + RPR * k;
        const int ly = row % BY, lz = row / BY;
        const int gy = gy0 + ly, gz = gz0 + lz;
        const bool ok = okx && row < NROW && (unsigned)gy < (unsigned)iy && (unsigned)gz < (unsigned)iz;
        okm |= ok ? (1u << k) : 0u;
        // node index within the volume: below 2^31 (the launchers check)
        const uint32_t node = ok ? (uint32_t)((gz * iy + gy) * ix + gx) : 0u;
        q[k] = *reinterpret_cast<const V*>(pe + (uint64_t)node * CIN);
    }
#pragma unroll
    for (int k = 0; k < ROUNDS; ++k) {
        const int row = r0 + RPR * k;
        if (r0 < RPR && row < NROW)
            *reinterpret_cast<V*>(&tile[row * (BX * CIN) + e * SLOT]) = ((okm >> k) & 1u) ? q[k] : V(0u);
    }
}

// Tile of workgroup blockIdx.x (XCD-aware order): volume and corner of its output box.
struct FTile {
    int vol, x0, y0, z0;
};
__device__ __forceinline__ FTile ftile_of(int tiles_x, int tiles_y, int tiles_z) {
    int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    FTile t;
    const int txi = b % tiles_x;
    b /= tiles_x;
    const int tyi = b % tiles_y;
    b /= tiles_y;
    const int tzi = b % tiles_z;
    t.vol = b / tiles_z;
    t.x0 = txi * FX;
    t.y0 = tyi * FY;
    t.z0 = tzi * FZ;
    return t;
}

// The 16-channel convolution of a staged FLX x FLY x FLZ tile (node-major, 32 bytes per
// node) for this wave's rows, and its epilogue.  w: this lane's 14 fragments (registers);
// bl: 16 biases in LDS.  Wave w computes the FNRY x FZ rows y0 + FNRY w + yy, z0 + rz.
// Input-row major: each B operand (16 nodes of one input row of the tile, an x pair or
// the x = 2 taps, one channel half per lane) is read from LDS once and multiplied into
// every row of the wave that reads it, with the chunk of its offset, so the wave reads 56
// operands for its 112 products.  Every row still receives its chunks in order 0..13 (the
// loops run dz outer, dy inner), the same sums as one row at a time.
template <int MODE>   // 0 or 2
__device__ __forceinline__ void conv16_rows(const uint16_t* tile, const U4 (&w)[14], const float* bl,
                                            const ConvArgs& a, const FTile& t) {
    constexpr int NODE_B = 32, ROW_B = FLX * NODE_B, PLANE_B = FLY * ROW_B;
    static_assert(FNRY == 2 && FZ == 4, "the operand schedule below is written for 2 x 4 rows");
    static_assert((FNRY + 1) * ROW_B + (FZ + 1) * PLANE_B < 65536, "LDS immediate offsets are 16 bits");
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    const uint32_t hi = (uint32_t)(g >> 1);
    const char* tb = reinterpret_cast<const char*>(tile);
    const int ry0 = wv * FNRY;
    // lane's node (ry0, z 0, x j), channel half g & 1
    const uint32_t rbase = (uint32_t)((ry0 * FLX + j) * NODE_B + (g & 1) * 16);
    // per-kind bases: the second tap of the lane's group (hi) sits one node along x (x pairs),
    // one plane along z (chunks 9..11) or one row along y (chunk 12); chunk 13's groups 2, 3
    // carry zero weights and read the first tap
    const uint32_t bP = rbase + hi * NODE_B;
    const uint32_t bQ = rbase + 2 * NODE_B + hi * PLANE_B;
    const uint32_t bR = rbase + 2 * NODE_B + hi * ROW_B;
    const uint32_t bS = rbase + 2 * NODE_B;
    auto ld = [&](uint32_t base, int Y, int Z) -> U4 {
        return *reinterpret_cast<const U4*>(tb + base + (Y * ROW_B + Z * PLANE_B));
    };
    f32x4 acc[8];   // row yy * 4 + rz
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] = f32x4{0.f, 0.f, 0.f, 0.f};
    // x pairs: input row (Y, Z) feeds output row (yy, rz) with chunk 3 (Z - rz) + (Y - yy)
#pragma unroll
    for (int Z = 0; Z < FZ + 2; ++Z)
#pragma unroll
        for (int Y = 0; Y < FNRY + 2; ++Y) {
            const U4 b = ld(bP, Y, Z);
#pragma unroll
            for (int yy = 0; yy < FNRY; ++yy)
#pragma unroll
                for (int rz = 0; rz < FZ; ++rz) {
                    const int dy = Y - yy, dz = Z - rz;
                    if (dy >= 0 && dy <= 2 && dz >= 0 && dz <= 2)
                        acc[yy * FZ + rz] = mfma_bf16(w[3 * dz + dy], b, acc[yy * FZ + rz]);
                }
        }
    // x = 2 taps of planes dz 0 and 1: input row (Y, rz) feeds row (yy, rz) with chunk 9 + (Y - yy)
#pragma unroll
    for (int rz = 0; rz < FZ; ++rz)
#pragma unroll
        for (int Y = 0; Y < FNRY + 2; ++Y) {
            const U4 b = ld(bQ, Y, rz);
#pragma unroll
            for (int yy = 0; yy < FNRY; ++yy) {
                const int dy = Y - yy;
                if (dy >= 0 && dy <= 2) acc[yy * FZ + rz] = mfma_bf16(w[9 + dy], b, acc[yy * FZ + rz]);
            }
        }
    // chunks 12 and 13
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int yy = r / FZ, rz = r % FZ;
        acc[r] = mfma_bf16(w[12], ld(bR, yy, rz + 2), acc[r]);
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const int yy = r / FZ, rz = r % FZ;
        acc[r] = mfma_bf16(w[13], ld(bS, yy + 2, rz + 2), acc[r]);
    }

    const int ox = t.x0 + j;
    if (ox >= a.ox) return;
    const float bias[4] = {bl[4 * g], bl[4 * g + 1], bl[4 * g + 2], bl[4 * g + 3]};
    const int64_t pstride = (int64_t)a.oy * a.ox * 16;
#pragma unroll
    for (int yy = 0; yy < FNRY; ++yy) {
        const int oy = t.y0 + ry0 + yy;
        if (oy >= a.oy) break;
        // output of node (z0 + rz, oy, ox): one pointer, advanced by a plane per row
        const int64_t e0 = (int64_t)t.vol * a.out_vstride + (((int64_t)t.z0 * a.oy + oy) * a.ox + ox) * 16 + 4 * g;
        uint16_t* oh = reinterpret_cast<uint16_t*>(a.out) + e0;
        const uint16_t* mh = a.mask + e0;
#pragma unroll
        for (int rz = 0; rz < FZ; ++rz) {
            if (t.z0 + rz >= a.oz) break;
            const f32x4 v = acc[yy * FZ + rz];
            uint2 st;
            if (MODE == 0) {
                st.x = pack2bf(fmaxf(v[0] + bias[0], 0.f), fmaxf(v[1] + bias[1], 0.f));
                st.y = pack2bf(fmaxf(v[2] + bias[2], 0.f), fmaxf(v[3] + bias[3], 0.f));
            } else {
                const uint2 m = *reinterpret_cast<const uint2*>(mh);
                mh += pstride;
                st.x = pack2bf(bf2f(m.x) > 0.f ? v[0] : 0.f, bf2f(m.x >> 16) > 0.f ? v[1] : 0.f);
                st.y = pack2bf(bf2f(m.y) > 0.f ? v[2] : 0.f, bf2f(m.y >> 16) > 0.f ? v[3] : 0.f);
            }
            *reinterpret_cast<uint2*>(oh) = st;
            oh += pstride;
        }
    }
}

// Layer 1 (2 -> 16 channels, ReLU, bf16) of NODES nodes of a box of BX x BY x BZ output
// nodes, written into a 16-channel LDS tile (node-major, 32 bytes per node).  `feat` is the
// staged 2-channel input box, (BX + 2) x (BY + 2) x (BZ + 2).  16 consecutive box nodes per
// product (a lane's node index picks its own input address); 2 chunks of 4 taps x 2
// channels per lane, in layer 1's k order (l1_tap); each wave takes groups w, w + 8, ..., two at a time.  w0: the layer's
// 2 fragments of this lane; b0: the biases of this lane's 4 output channels.  The same
// chunks, operands and rounding as k_conv<2, 0>, so the values are those it stores.
template <int BX, int BY, int BZ>
__device__ __forceinline__ void layer1_to_lds(const uint16_t* feat, uint16_t* out, const U4 (&w0)[2],
                                              const float (&b0)[4]) {
    constexpr int NODES = BX * BY * BZ, NGRP = (NODES + 15) / 16;
    constexpr int IX = BX + 2, IY = BY + 2;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    // per-lane offsets (in input nodes) of the 4 taps of each chunk: tap l1_read_tap(c, g, q)
    int toff[8];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int tt[4];
#pragma unroll
            for (int gg = 0; gg < 4; ++gg) {
                const int t = l1_read_tap(c, gg, q);
                tt[gg] = ((t / 9) * IY + (t / 3) % 3) * IX + t % 3;
            }
            toff[c * 4 + q] = (g & 2) ? ((g & 1) ? tt[3] : tt[2]) : ((g & 1) ? tt[1] : tt[0]);
        }
    const uint32_t* fw = reinterpret_cast<const uint32_t*>(feat);
#pragma unroll 1
    for (int grp = wv; grp < NGRP; grp += 2 * (FTHREADS / 64)) {
        int n[2], base[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            n[h] = (grp + h * (FTHREADS / 64)) * 16 + j;
            const int m = n[h] < NODES ? n[h] : NODES - 1;
            const int lx = m % BX, r = m / BX;
            base[h] = ((r / BY) * IY + r % BY) * IX + lx;
        }
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            U4 b0v, b1v;
            b0v.x = fw[base[0] + toff[c * 4 + 0]];
            b0v.y = fw[base[0] + toff[c * 4 + 1]];
            b0v.z = fw[base[0] + toff[c * 4 + 2]];
            b0v.w = fw[base[0] + toff[c * 4 + 3]];
            b1v.x = fw[base[1] + toff[c * 4 + 0]];
            b1v.y = fw[base[1] + toff[c * 4 + 1]];
            b1v.z = fw[base[1] + toff[c * 4 + 2]];
            b1v.w = fw[base[1] + toff[c * 4 + 3]];
            acc0 = mfma_bf16(w0[c], b0v, acc0);
            acc1 = mfma_bf16(w0[c], b1v, acc1);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const f32x4 v = h ? acc1 : acc0;
            if (n[h] < NODES) {
                uint2 st;
                st.x = pack2bf(fmaxf(v[0] + b0[0], 0.f), fmaxf(v[1] + b0[1], 0.f));
                st.y = pack2bf(fmaxf(v[2] + b0[2], 0.f), fmaxf(v[3] + b0[3], 0.f));
                *reinterpret_cast<uint2*>(&out[n[h] * 16 + 4 * g]) = st;
            }
        }
    }
}

// Forward / bwd-data convolution of one FX x FY x FZ output box per workgroup of 8 waves:
// the input tile (halo 2) and the weight fragments staged in LDS (76.5 KB with 16 input
// channels: two workgroups, 16 waves, per compute unit).
template <int CIN, int MODE>
__global__ __launch_bounds__(FTHREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_conv(ConvArgs a) {
    constexpr int NCH = CIN == 16 ? 14 : 2;      // 32-wide k chunks: ceil(27 * CIN / 32)
    constexpr int NV = FLZ * FLY * FLX;          // nodes of the staged tile
    __shared__ __align__(16) uint16_t tile[NV * CIN];
    __shared__ __align__(16) U4 wl[CIN == 16 ? 1 : NCH * 64];   // layer 1 only
    __shared__ float bl[16];

    const FTile t = ftile_of(a.tiles_x, a.tiles_y, a.tiles_z);
    if (threadIdx.x < 16) bl[threadIdx.x] = (MODE != 2 && (int)threadIdx.x < a.cout) ? a.bias[threadIdx.x] : 0.f;
    if constexpr (CIN == 16) {
        const int lane = threadIdx.x & 63;
        U4 w[14];
#pragma unroll
        for (int c = 0; c < 14; ++c) w[c] = reinterpret_cast<const U4*>(a.wfrag)[c * 64 + lane];
        stage_box<CIN, FLX, FLY, FLZ>(a.in + (int64_t)t.vol * a.in_vstride, a.ix, a.iy, a.iz, t.x0 + a.off,
                                      t.y0 + a.off, t.z0 + a.off, tile);
        __syncthreads();
        conv16_rows<MODE>(tile, w, bl, a, t);
    } else {
        for (int u = threadIdx.x; u < NCH * 64; u += FTHREADS) wl[u] = reinterpret_cast<const U4*>(a.wfrag)[u];
        stage_box<CIN, FLX, FLY, FLZ>(a.in + (int64_t)t.vol * a.in_vstride, a.ix, a.iy, a.iz, t.x0 + a.off,
                                      t.y0 + a.off, t.z0 + a.off, tile);
        // layer 1 on its own (training keeps its output): FX x FY x FZ outputs from the tile
        U4 w0[2];
        float b0[4];
        const int lane = threadIdx.x & 63, g = lane >> 4;
        __syncthreads();
        w0[0] = wl[lane];
        w0[1] = wl[64 + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r) b0[r] = bl[4 * g + r];
        // compute into LDS rows, then copy out: reuse the rows of the output box
        __shared__ __align__(16) uint16_t ob[FX * FY * FZ * 16];
        layer1_to_lds<FX, FY, FZ>(tile, ob, w0, b0);
        __syncthreads();
        // store the box: 2 x 16 bytes per node, node-major as the output volume
        for (int u = threadIdx.x; u < FX * FY * FZ * 2; u += FTHREADS) {
            const int n = u >> 1, h = u & 1;
            const int lx = n % FX, r = n / FX, ly = r % FY, lz = r / FY;
            const int ox = t.x0 + lx, oy = t.y0 + ly, oz = t.z0 + lz;
            if (ox < a.ox && oy < a.oy && oz < a.oz)
                *reinterpret_cast<U4*>(reinterpret_cast<uint16_t*>(a.out) + (int64_t)t.vol * a.out_vstride +
                                       (((int64_t)oz * a.oy + oy) * a.ox + ox) * 16 + h * 8) =
                    *reinterpret_cast<const U4*>(&ob[n * 16 + h * 8]);
        }
    }
}

// Layers 1 and 2 fused (features -> 16 -> 16 channels, ReLU after each): the workgroup
// stages the (FX + 4) x (FY + 4) x (FZ + 4) feature box, computes layer 1 on the
// FLX x FLY x FLZ nodes that layer 2 reads into LDS (halo nodes recomputed by the
// neighbouring workgroups), then runs layer 2 as k_conv<16, 0> does.  Layer 1's output
// never leaves the chip.
struct Conv12Args {
    ConvArgs l2;                 // layer 2 (in unused: layer 1's output is the tile)
    const uint16_t* feat;        // padded features, 2 channels
    int fz, fy, fx;              // feature volume shape
    int64_t feat_vstride;
    const void* wfrag1;          // layer 1 fragments (2 chunks)
    const float* bias1;
};

__global__ __launch_bounds__(FTHREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_conv12(Conv12Args a) {
    constexpr int NV = FLZ * FLY * FLX;
    constexpr int FB = (FX + 4) * (FY + 4) * (FZ + 4);   // feature box nodes
    __shared__ __align__(16) uint16_t tile[NV * 16];
    __shared__ __align__(16) uint16_t fb[FB * 2];
    __shared__ float bl[16];

    const ConvArgs& l2 = a.l2;
    const FTile t = ftile_of(l2.tiles_x, l2.tiles_y, l2.tiles_z);
    const int lane = threadIdx.x & 63, g = lane >> 4;
    U4 w2[14];
#pragma unroll
    for (int c = 0; c < 14; ++c) w2[c] = reinterpret_cast<const U4*>(l2.wfrag)[c * 64 + lane];
    U4 w0[2];
    w0[0] = reinterpret_cast<const U4*>(a.wfrag1)[lane];
    w0[1] = reinterpret_cast<const U4*>(a.wfrag1)[64 + lane];
    float b0[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) b0[r] = a.bias1[4 * g + r];
    if (threadIdx.x < 16) bl[threadIdx.x] = (int)threadIdx.x < l2.cout ? l2.bias[threadIdx.x] : 0.f;
    stage_box<2, FX + 4, FY + 4, FZ + 4>(a.feat + (int64_t)t.vol * a.feat_vstride, a.fx, a.fy, a.fz, t.x0, t.y0,
                                         t.z0, fb);
    __syncthreads();
    layer1_to_lds<FLX, FLY, FLZ>(fb, tile, w0, b0);
    __syncthreads();
    conv16_rows<0>(tile, w2, bl, l2, t);
}

// The last layer (16 channels -> 1, no ReLU, FP32 out) by shifts.  One output channel would
// use 1 of the 16 rows of a product; instead the rows are the 9 (dz, dy) shifts: for an
// input row (y, z) of the staged tile, D[s][x] = sum over dx, ci of w[dz, dy, dx, ci]
// a[y, z, x + dx, ci] (two products: the x pair, then x = 2) is the contribution of that
// input row to output row (y - dy, z - dz).  Lane (x, g) holds shifts s = 4 g .. 4 g + 3 of
// each D; it adds those that belong to its wave's 8 output rows (a multiply by its group's
// 0/1 selector keeps the instruction stream uniform), and the 4 lane groups are summed at
// the end.  48 products per wave for 8 rows of 16 nodes, against 112 one channel at a time.
__global__ __launch_bounds__(FTHREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_conv_last(ConvArgs a) {
    constexpr int NV = FLZ * FLY * FLX;
    constexpr int NODE_B = 32, ROW_B = FLX * NODE_B, PLANE_B = FLY * ROW_B;
    static_assert(FNRY == 2 && FZ == 4, "the schedule below is written for 2 x 4 rows");
    static_assert((FNRY + 1) * ROW_B + (FZ + 1) * PLANE_B < 65536, "LDS immediate offsets are 16 bits");
    __shared__ __align__(16) uint16_t tile[NV * 16];

    const FTile t = ftile_of(a.tiles_x, a.tiles_y, a.tiles_z);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    const U4 wP = reinterpret_cast<const U4*>(a.wfrag)[lane];
    const U4 wS = reinterpret_cast<const U4*>(a.wfrag)[64 + lane];
    const float bias = a.bias[0];
    stage_box<16, FLX, FLY, FLZ>(a.in + (int64_t)t.vol * a.in_vstride, a.ix, a.iy, a.iz, t.x0, t.y0, t.z0, tile);
    __syncthreads();

    const uint32_t hi = (uint32_t)(g >> 1);
    const char* tb = reinterpret_cast<const char*>(tile);
    const int ry0 = wv * FNRY;
    const uint32_t rbase = (uint32_t)((ry0 * FLX + j) * NODE_B + (g & 1) * 16);
    const uint32_t bP = rbase + hi * NODE_B;   // x pair: groups 2, 3 one node along x
    const uint32_t bS = rbase + 2 * NODE_B;    // x = 2 (groups 2, 3: zero weights)
    auto ld = [&](uint32_t base, int Y, int Z) -> U4 {
        return *reinterpret_cast<const U4*>(tb + base + (Y * ROW_B + Z * PLANE_B));
    };
    const float sel[3] = {g == 0 ? 1.f : 0.f, g == 1 ? 1.f : 0.f, g == 2 ? 1.f : 0.f};
    float acc[8];   // row yy * 4 + rz, this lane group's share
#pragma unroll
    for (int r = 0; r < 8; ++r) acc[r] = 0.f;
#pragma unroll
    for (int Z = 0; Z < FZ + 2; ++Z)
#pragma unroll
        for (int Y = 0; Y < FNRY + 2; ++Y) {
            f32x4 d = mfma_bf16(wP, ld(bP, Y, Z), f32x4{0.f, 0.f, 0.f, 0.f});
            d = mfma_bf16(wS, ld(bS, Y, Z), d);
#pragma unroll
            for (int yy = 0; yy < FNRY; ++yy)
#pragma unroll
                for (int rz = 0; rz < FZ; ++rz) {
                    const int dy = Y - yy, dz = Z - rz;
                    if (dy >= 0 && dy <= 2 && dz >= 0 && dz <= 2) {
                        const int sh = 3 * dz + dy;
                        acc[yy * FZ + rz] = __builtin_fmaf(d[sh & 3], sel[sh >> 2], acc[yy * FZ + rz]);
                    }
                }
        }
    // sum the four lane groups (group 3 holds zeros): g and g ^ 1, then g and g ^ 2
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        acc[r] += __shfl_xor(acc[r], 16);
        acc[r] += __shfl_xor(acc[r], 32);
    }
    const int ox = t.x0 + j;
    if (g != 0 || ox >= a.ox) return;
    const int64_t pstride = (int64_t)a.oy * a.ox;
#pragma unroll
    for (int yy = 0; yy < FNRY; ++yy) {
        const int oy = t.y0 + ry0 + yy;
        if (oy >= a.oy) break;
        float* of = reinterpret_cast<float*>(a.out) + (int64_t)t.vol * a.out_vstride +
                    (((int64_t)t.z0 * a.oy + oy) * a.ox + ox);
#pragma unroll
        for (int rz = 0; rz < FZ; ++rz) {
            if (t.z0 + rz >= a.oz) break;
            *of = acc[yy * FZ + rz] + bias;
            of += pstride;
        }
    }
}

// ---- bwd-weight --------------------------------------------------------------------------
//
// Per workgroup: one TX x TY x TZ tile of output nodes of one volume.  For each tap,
// D[co][ci] = sum over the tile's nodes of g[node][co] * x[node + tap][ci]  (k = nodes).
// Both operands are staged planar in LDS (channel-major) so that 8 consecutive nodes of
// one channel are contiguous.  Output: partial[block][tap][co][ci] and the bias partial
// sum_node g[node][co] at partial[block][27 * 256 + co].
template <int CIN>
__global__ __launch_bounds__(NTHREADS) void k_conv_bwdw(BwdWArgs a) {
    constexpr int NX = LZ * LY * LX, NG = TZ * TY * TX;
    __shared__ __align__(16) uint16_t xs[CIN * NX];
    __shared__ __align__(16) uint16_t gs[16 * NG];
    __shared__ float bsum[NTHREADS];

    int b = blockIdx.x;
    const int txi = b % a.tiles_x;
    b /= a.tiles_x;
    const int tyi = b % a.tiles_y;
    b /= a.tiles_y;
    const int tzi = b % a.tiles_z;
    const int vol = b / a.tiles_z;
    const int x0 = txi * TX, y0 = tyi * TY, z0 = tzi * TZ;
    const uint16_t* xin = a.x + (int64_t)vol * a.x_vstride;
    const uint16_t* gin = a.g + (int64_t)vol * a.g_vstride;

    for (int v = threadIdx.x; v < NX; v += NTHREADS) {
        const int lx = v % LX, ly = (v / LX) % LY, lz = v / (LX * LY);
        const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        const bool in = gx < a.ix && gy < a.iy && gz < a.iz;
        const int64_t src = (((int64_t)gz * a.iy + gy) * a.ix + gx) * CIN;
        if (CIN == 16) {
            U4 q0 = {0u, 0u, 0u, 0u}, q1 = {0u, 0u, 0u, 0u};
            if (in) {
                q0 = *reinterpret_cast<const U4*>(xin + src);
                q1 = *reinterpret_cast<const U4*>(xin + src + 8);
            }
            const uint32_t w8[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                xs[(2 * c) * NX + v] = (uint16_t)(w8[c] & 0xFFFFu);
                xs[(2 * c + 1) * NX + v] = (uint16_t)(w8[c] >> 16);
            }
        } else {
            uint32_t q = in ? *reinterpret_cast<const uint32_t*>(xin + src) : 0u;
            xs[v] = (uint16_t)(q & 0xFFFFu);
            xs[NX + v] = (uint16_t)(q >> 16);
        }
    }
    for (int v = threadIdx.x; v < NG; v += NTHREADS) {
        const int tx = v % TX, ty = (v / TX) % TY, tz = v / (TX * TY);
        const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
        U4 q0 = {0u, 0u, 0u, 0u}, q1 = {0u, 0u, 0u, 0u};
        if (gx < a.ox && gy < a.oy && gz < a.oz) {
            const int64_t src = (((int64_t)gz * a.oy + gy) * a.ox + gx) * 16;
            q0 = *reinterpret_cast<const U4*>(gin + src);
            q1 = *reinterpret_cast<const U4*>(gin + src + 8);
        }
        const uint32_t w8[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            gs[(2 * c) * NG + v] = (uint16_t)(w8[c] & 0xFFFFu);
            gs[(2 * c + 1) * NG + v] = (uint16_t)(w8[c] >> 16);
        }
    }
    __syncthreads();

    float* part = a.partial + (int64_t)blockIdx.x * CNN_PARTIAL_STRIDE;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 15, g = lane >> 4;
    for (int t = wv; t < 27; t += NTHREADS / 64) {
        int dz, dy, dx;
        tap_xyz(t, dz, dy, dx);
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int c = 0; c < NG / 32; ++c) {
            const int row = 2 * c + (g >> 1);           // row = tz * TY + ty
            const int ty = row % TY, tz = row / TY, xo = 8 * (g & 1);
            const U4 aop = *reinterpret_cast<const U4*>(&gs[j * NG + row * TX + xo]);
            U4 bop = {0u, 0u, 0u, 0u};
            if (j < CIN) {
                const uint16_t* p = &xs[j * NX + ((tz + dz) * LY + ty + dy) * LX + xo + dx];
                bop.x = (uint32_t)p[0] | ((uint32_t)p[1] << 16);
                bop.y = (uint32_t)p[2] | ((uint32_t)p[3] << 16);
                bop.z = (uint32_t)p[4] | ((uint32_t)p[5] << 16);
                bop.w = (uint32_t)p[6] | ((uint32_t)p[7] << 16);
            }
            acc = mfma_bf16(aop, bop, acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) part[t * 256 + (4 * g + r) * 16 + j] = acc[r];
    }
    // bias: sum over the tile of g[node][co]; 16 threads per channel
    {
        const int co = threadIdx.x & 15, q = threadIdx.x >> 4;
        float s = 0.f;
        for (int v = q; v < NG; v += NTHREADS / 16) s += bf2f(gs[co * NG + v]);
        bsum[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x < 16) {
            float t = 0.f;
            for (int k = 0; k < NTHREADS / 16; ++k) t += bsum[k * 16 + threadIdx.x];
            part[27 * 256 + threadIdx.x] = t;
        }
    }
}

// Sum of the per-workgroup partials into the flat gradient of one layer (FP32, the
// parameter order W[co][ci][tap], b[co]).
__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ partial, int nblocks, int cin,
                                                     int cout, float* __restrict__ grad) {
    const int nw = cout * cin * 27;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nw + cout) return;
    int src;
    if (p < nw) {
        const int co = p / (cin * 27), ci = (p / 27) % cin, t = p % 27;
        src = t * 256 + co * 16 + ci;
    } else {
        src = 27 * 256 + (p - nw);
    }
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += partial[(int64_t)b * CNN_PARTIAL_STRIDE + src];
    grad[p] = s;
}

// Loss: r = y - log(gamma + 0.01) at nodes with gamma >= 0; output gradient
// bf16(scale * r) into channel 0 of a 16-channel tensor (other channels 0), and one
// partial sum of r^2 per workgroup.
__global__ __launch_bounds__(256) void k_loss(const float* __restrict__ y, const float* __restrict__ gamma,
                                              int64_t n, float scale, uint16_t* __restrict__ gout,
                                              float* __restrict__ loss_part) {
    __shared__ float red[256];
    float s = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float gm = gamma[i];
        float r = 0.f;
        if (gm >= 0.f) r = y[i] - logf(gm + 0.01f);
        s += r * r;
        U4 q0 = {(uint32_t)f2bf(scale * r), 0u, 0u, 0u}, q1 = {0u, 0u, 0u, 0u};
        *reinterpret_cast<U4*>(gout + i * 16) = q0;
        *reinterpret_cast<U4*>(gout + i * 16 + 8) = q1;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Adam with bias correction (c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)).
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ theta, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ grad, int n, float lr,
                                              float beta1, float beta2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = grad[i];
    const float mi = beta1 * m[i] + (1.f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    theta[i] = theta[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Fragments of one layer from the FP32 parameters.  Lane l of chunk c holds row l % 16
// and k = 32 c + 8 (l / 16) + e, e = 0..7.
//   forward, 2 channels : row = co; k = 32 c + 8 g + 2 q + ci, tap l1_tap(c, g, q)
//   forward, 16 channels: row = co; k = 16 h + ci, tap chunk_tap(c, h)
//   backward: row = ci; k = 16 h + co, tap' = chunk_tap(c, h) of the flipped kernel
//             (tap 26 - tap', bwd-data)
//   bwd == 2, the last layer (16 -> 1) by shifts: row = s = 3 dz + dy (rows 9..15 zero);
//             chunk 0: k = 16 dx + ci, dx = 0, 1; chunk 1: k = ci, dx = 2 (k 16..31 zero)
__global__ __launch_bounds__(64) void k_pack(const float* __restrict__ w, int cin, int cout, int bwd, int nch,
                                             uint16_t* __restrict__ frag) {
    const int c = blockIdx.x, lane = threadIdx.x;
    if (c >= nch) return;
    const int row = lane & 15, g = lane >> 4;
    uint16_t h[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = 32 * c + 8 * g + e;
        float val = 0.f;
        if (bwd == 2) {
            // one output channel, rows = the 9 (dz, dy) shifts s = 3 dz + dy: chunk 0 holds
            // dx = k / 16 (0, 1), chunk 1 dx = 2 (k < 16); channel k % 16
            const int kl = k & 31;   // k within the chunk
            const int dx = c == 0 ? (kl >> 4) : (kl < 16 ? 2 : 3);
            if (row < 9 && dx < 3) val = w[(k & 15) * 27 + 9 * (row / 3) + 3 * (row % 3) + dx];
        } else if (!bwd) {
            // 16 input channels: the chunk table; 2: layer 1's k order
            const int t = cin == 16 ? chunk_tap(c, (k >> 4) & 1) : (cin == 2 ? l1_tap(c, g, e >> 1) : 27);
            const int ci = k % cin;
            if (t < 27 && row < cout) val = w[(row * cin + ci) * 27 + t];
        } else {
            const int tp = chunk_tap(c, (k >> 4) & 1), co = k % 16;
            if (tp < 27 && co < cout && row < cin) val = w[(co * cin + row) * 27 + (26 - tp)];
        }
        h[e] = f2bf(val);
    }
    U4 q;
    q.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
    q.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
    q.z = (uint32_t)h[4] | ((uint32_t)h[5] << 16);
    q.w = (uint32_t)h[6] | ((uint32_t)h[7] << 16);
    reinterpret_cast<U4*>(frag)[c * 64 + lane] = q;
}

// Features on the grid padded by 4: f0 = D_r * fl32(1/Dmax), f1 = (D_e - D_r) * inv_dd,
// both bf16; 0 outside the grid.  Dmax and inv_dd come from the prep's scalars.
__global__ __launch_bounds__(256) void k_features(const float* __restrict__ ref, const float* __restrict__ ev,
                                                  int nz, int ny, int nx, const Scalars* __restrict__ sc,
                                                  uint16_t* __restrict__ feat) {
    const int pz = nz + 8, py = ny + 8, px = nx + 8;
    const int64_t total = (int64_t)pz * py * px;
    const float dmax = ord_to_float(sc->dmax_ord);
    const float inv_max = 1.0f / dmax;
    const float inv_dd = sc->inv_dd;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int x = (int)(i % px) - 4, y = (int)((i / px) % py) - 4, z = (int)(i / ((int64_t)px * py)) - 4;
        uint32_t q = 0u;
        if (x >= 0 && x < nx && y >= 0 && y < ny && z >= 0 && z < nz) {
            const int64_t n = ((int64_t)z * ny + y) * nx + x;
            const float r = ref[n], e = ev[n];
            q = (uint32_t)f2bf(r * inv_max) | ((uint32_t)f2bf((e - r) * inv_dd) << 16);
        }
        reinterpret_cast<uint32_t*>(feat)[i] = q;
    }
}

// Features of the pair average-pooled 2x2x2 onto the coarse grid (cz, cy, cx) = ceil(n / 2),
// padded by 4: coarse node c takes the mean of the fine nodes 2c and 2c + 1 per axis that lie
// in the grid (fewer at an odd edge); f0 and f1 as in k_features, with the fine grid's Dmax
// and inv_dd.  One thread per padded coarse node, 32-bit index arithmetic (the launcher
// bounds the padded coarse volume below 2^31); the two fine nodes of a pair along x are one
// 8-byte load when nx is even and both volumes start 8-byte aligned (every pair then is),
// two loads otherwise.  The sums run in the same order either way.
__global__ __launch_bounds__(256) void k_features_pool2(const float* __restrict__ ref, const float* __restrict__ ev,
                                                        int nz, int ny, int nx, const Scalars* __restrict__ sc,
                                                        uint16_t* __restrict__ feat) {
    const int cz = (nz + 1) >> 1, cy = (ny + 1) >> 1, cx = (nx + 1) >> 1;
    const uint32_t pz = cz + 8, py = cy + 8, px = cx + 8;
    const uint32_t total = pz * py * px;
    const float dmax = ord_to_float(sc->dmax_ord);
    const float inv_max = 1.0f / dmax;
    const float inv_dd = sc->inv_dd;
    const bool even = (nx & 1) == 0 && ((reinterpret_cast<uintptr_t>(ref) | reinterpret_cast<uintptr_t>(ev)) & 7) == 0;
    for (uint32_t i = blockIdx.x * 256u + threadIdx.x; i < total; i += gridDim.x * 256u) {
        const uint32_t row = i / px;
        const int x = (int)(i - row * px) - 4, y = (int)(row % py) - 4, z = (int)(row / py) - 4;
        uint32_t q = 0u;
        if (x >= 0 && x < cx && y >= 0 && y < cy && z >= 0 && z < cz) {
            float sr = 0.f, se = 0.f;
            int cnt = 0;
            const int fx = 2 * x;
            const bool two = fx + 1 < nx;
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy) {
                    const int fz = 2 * z + dz, fy = 2 * y + dy;
                    if (fz < nz && fy < ny) {
                        const int64_t n = ((int64_t)fz * ny + fy) * nx + fx;
                        float r0, r1, e0, e1;
                        if (even) {
                            const float2 rr = *reinterpret_cast<const float2*>(ref + n);
                            const float2 ee = *reinterpret_cast<const float2*>(ev + n);
                            r0 = rr.x, r1 = rr.y, e0 = ee.x, e1 = ee.y;
                        } else {
                            r0 = ref[n], e0 = ev[n];
                            r1 = two ? ref[n + 1] : 0.f;
                            e1 = two ? ev[n + 1] : 0.f;
                        }
                        sr += r0;
                        se += e0;
                        ++cnt;
                        if (two) {
                            sr += r1;
                            se += e1;
                            ++cnt;
                        }
                    }
                }
            const float r = sr / (float)cnt, e = se / (float)cnt;
            q = pack2bf(r * inv_max, (e - r) * inv_dd);
        }
        reinterpret_cast<uint32_t*>(feat)[i] = q;
    }
}

// Trilinear weights of fine node index p on a coarse axis of c nodes whose node k sits at
// fine position 2k + 1/2: coarse position u = (p - 1/2) / 2 clamped to [0, c - 1].
__device__ __forceinline__ void pool2_axis(int p, int c, int& i0, int& i1, float& t) {
    float u = 0.5f * (float)p - 0.25f;
    u = fminf(fmaxf(u, 0.0f), (float)(c - 1));
    i0 = min((int)u, c - 1);
    i1 = min(i0 + 1, c - 1);
    t = u - (float)i0;
}

// y at listed fine nodes (grid nz x ny x nx) from the coarse network output yc (grid
// ceil(n / 2)): exp(yc) = gamma_hat + 0.01 interpolated trilinearly, y = its log.
__global__ __launch_bounds__(256) void k_cnn_upsample(const float* __restrict__ yc, int nz, int ny, int nx,
                                                      const uint32_t* __restrict__ nodes,
                                                      const uint32_t* __restrict__ count, float* __restrict__ y,
                                                      uint32_t* __restrict__ key) {
    const int cz = (nz + 1) >> 1, cy = (ny + 1) >> 1, cx = (nx + 1) >> 1;
    const uint32_t M = *count;
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < M; i += gridDim.x * 256) {
        const int node = (int)nodes[i];
        const int x = node % nx, yy = (node / nx) % ny, z = node / (nx * ny);
        int z0, z1, y0, y1, x0, x1;
        float tz, ty, tx;
        pool2_axis(z, cz, z0, z1, tz);
        pool2_axis(yy, cy, y0, y1, ty);
        pool2_axis(x, cx, x0, x1, tx);
        float g[8];   // corner k: z from bit 2, y from bit 1, x from bit 0
#pragma unroll
        for (int k = 0; k < 8; ++k)
            g[k] = expf(yc[((int64_t)(k & 4 ? z1 : z0) * cy + (k & 2 ? y1 : y0)) * cx + (k & 1 ? x1 : x0)]);
        const float v00 = g[0] + tx * (g[1] - g[0]), v01 = g[2] + tx * (g[3] - g[2]);
        const float v10 = g[4] + tx * (g[5] - g[4]), v11 = g[6] + tx * (g[7] - g[6]);
        const float v0 = v00 + ty * (v01 - v00), v1 = v10 + ty * (v11 - v10);
        const float v = v0 + tz * (v1 - v0);
        const float yv = logf(v);
        y[i] = yv;
        if (key) key[i] = f2u(fmaxf(expf(yv) - 0.01f, 0.0f));
    }
}

// ---- the network at listed nodes only ------------------------------------------------
//
// One workgroup per node (grid-stride over the list): the node's 9x9x9 feature patch is
// staged in LDS, then layer 1 (7^3 outputs), layer 2 (5^3), layer 3 (3^3) run as the same
// implicit GEMM on the matrix cores with their outputs kept in LDS, and layer 4 (one
// output, 432 products) is a block reduction.  Same features, same bf16 rounding points
// and the same layer arithmetic as the dense pass, so the value at a node is what the dense
// network gives there (up to the order of the FP32 sums).
struct TailCnnArgs {
    const float* ref;
    const float* ev;
    int nx, ny, nz;
    const Scalars* sc;
    const uint32_t* nodes;      // node index per list entry
    const uint32_t* count;      // list length (device)
    const uint16_t* frag[3];    // forward fragments of layers 0..2
    const float* bias[3];
    const float* w4;            // layer 3 weights W[0][ci][tap] (FP32 master copy)
    const float* b4;            // layer 3 bias
    float* y;                   // output per list entry: log(gamma_hat + 0.01)
    uint32_t* key;              // optional: bits of gamma_hat per list entry (sort key)
};

// One wave evaluates the network at one listed node at a time, from its own 9^3 feature
// patch: 7^3, 5^3 and 3^3 hidden activations, then the single output.  The wave holds the
// fragments of the first three layers in registers for all its nodes; its LDS is two
// buffers that the layers use in turn (features and 5^3 in Y, 7^3 and 3^3 in X), about
// 15 KB.  The fragments take about 120 VGPRs, so two waves fit a SIMD (eight per compute
// unit) without spills; they hide one another's gather and LDS latency.
//
// The hidden activations are stored in two channel planes (channels 0-7, then 8-15, 16
// bytes per node in each), so the 16 lanes of a B-operand group read 16 consecutive nodes'
// records of one plane: 256 contiguous bytes, every bank once.
constexpr int TAIL_THREADS = 64;
constexpr int TAIL_XP = 343 * 8;         // plane stride of X (bf16 elements)
constexpr int TAIL_YP = 125 * 8;         // plane stride of Y
constexpr int TAIL_X_ELEMS = 2 * TAIL_XP;
constexpr int TAIL_Y_ELEMS = 2 * TAIL_YP;
static_assert(TAIL_Y_ELEMS >= 729 * 2, "Y holds the 9^3 x 2 features");
constexpr int TAIL_GATHER = (729 + 63) / 64;

// Byte addresses from which this lane reads the 14 chunks of a 16-channel layer for the
// output node whose input-patch base index is `base`: the lane's k slice is 8 channels
// (plane g & 1) of tap chunk_tap(c, g >> 1), and the tap's offset is a per-lane term (the
// h = g >> 1 half of the x pair, dz pair or dy pair) plus a constant per chunk.
template <int IN_E, int PLANE>
struct TapBases {
    uint32_t a, b, c, d;
    __device__ __forceinline__ TapBases(uint32_t base, uint32_t g) {
        const uint32_t p = ((g & 1u) * PLANE + base * 8u) * 2u, h = g >> 1;
        a = p + h * 16u;                   // chunks 0..8: (dz, dy, h)
        b = p + h * (IN_E * IN_E * 16u);   // chunks 9..11: (h, dy, 2)
        c = p + h * (IN_E * 16u);          // chunk 12: (2, h, 2)
        d = p;                             // chunk 13: (2, 2, 2), both halves
    }
    template <int C>
    __device__ __forceinline__ U4 load(const char* lds) const {
        constexpr uint32_t off = C < 9 ? ((C / 3) * IN_E + C % 3) * IN_E * 16u
                                       : (C < 12 ? ((C - 9) * IN_E + 2) * 16u
                                                 : (C == 12 ? (2 * IN_E * IN_E + 2) * 16u
                                                            : ((2 * IN_E + 2) * IN_E + 2) * 16u));
        const uint32_t v = C < 9 ? a : (C < 12 ? b : (C == 12 ? c : d));
        return *reinterpret_cast<const U4*>(lds + v + off);
    }
};
static_assert(chunk_tap(12, 1) == chunk_tap(12, 0) + 3 && chunk_tap(9, 1) == chunk_tap(9, 0) + 9 &&
                  chunk_tap(0, 1) == chunk_tap(0, 0) + 1 && chunk_tap(13, 0) == 26,
              "the per-lane tap terms follow the chunk table");

template <int C, int N, int IN_E, int PLANE>
__device__ __forceinline__ void tail_chunks(const char* in, const TapBases<IN_E, PLANE>& t0,
                                            const TapBases<IN_E, PLANE>& t1, const U4 (&wr)[14], f32x4& acc0,
                                            f32x4& acc1) {
    if constexpr (C < N) {
        const U4 b0 = t0.template load<C>(in);
        const U4 b1 = t1.template load<C>(in);
        acc0 = mfma_bf16(wr[C], b0, acc0);
        acc1 = mfma_bf16(wr[C], b1, acc1);
        tail_chunks<C + 1, N>(in, t0, t1, wr, acc0, acc1);
    }
}

// Store 16 output channels (this lane's 4 of node o) in the two-plane layout.
template <int OUT_PLANE>
__device__ __forceinline__ void tail_store(uint16_t* out, int o, uint32_t g, const f32x4& acc, const float (&bb)[4]) {
    uint2 st;
    st.x = pack2bf(fmaxf(acc[0] + bb[0], 0.f), fmaxf(acc[1] + bb[1], 0.f));
    st.y = pack2bf(fmaxf(acc[2] + bb[2], 0.f), fmaxf(acc[3] + bb[3], 0.f));
    *reinterpret_cast<uint2*>(&out[(g >> 1) * OUT_PLANE + o * 8 + (g & 1u) * 4]) = st;
}

// Output node o of a valid 3^3 convolution of an IN_E^3 patch -> the patch index of its
// (0, 0, 0) tap: o = (oz OUT_E + oy) OUT_E + ox  ->  (oz IN_E + oy) IN_E + ox
//   = o + (IN_E - OUT_E) (q + IN_E oz), q = o / OUT_E = oz OUT_E + oy.
template <int IN_E, int OUT_E>
__device__ __forceinline__ uint32_t tail_base(uint32_t o) {
    const uint32_t q = div_small<OUT_E>(o);
    const uint32_t oz = div_small<OUT_E>(q);
    return o + (IN_E - OUT_E) * (q + IN_E * oz);
}

// Output nodes [0, OUT_E^3) of a valid 3^3 convolution (16 input channels) of the IN_E^3
// patch `in` into the OUT_E^3 patch `out` (ReLU, bf16), 16 nodes per MFMA group.  Two groups
// are computed together so that their two accumulation chains alternate on the matrix core.
template <int IN_E, int OUT_E, int IN_PLANE, int OUT_PLANE>
__device__ __forceinline__ void tail_layer16(const uint16_t* __restrict__ in, uint16_t* __restrict__ out,
                                             const U4 (&wr)[14], const float* __restrict__ bias) {
    constexpr int NOUT = OUT_E * OUT_E * OUT_E;
    constexpr int NGRP = (NOUT + 15) / 16;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t j = lane & 15, g = lane >> 4;
    float bb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) bb[r] = bias[4 * g + r];
    const char* inb = reinterpret_cast<const char*>(in);
#pragma unroll 2   // two group pairs in flight: their reads overlap the other pair's products
    for (int grp = 0; grp < NGRP; grp += 2) {
        const int o0 = grp * 16 + j, o1 = o0 + 16;
        const bool v0 = o0 < NOUT, v1 = o1 < NOUT;   // (grp + 1 == NGRP: the second group is all invalid)
        const TapBases<IN_E, IN_PLANE> t0(tail_base<IN_E, OUT_E>(v0 ? o0 : NOUT - 1), g);
        const TapBases<IN_E, IN_PLANE> t1(tail_base<IN_E, OUT_E>(v1 ? o1 : NOUT - 1), g);
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
        tail_chunks<0, 14>(inb, t0, t1, wr, acc0, acc1);
        if (v0) tail_store<OUT_PLANE>(out, o0, g, acc0, bb);
        if (v1) tail_store<OUT_PLANE>(out, o1, g, acc1, bb);
    }
}

// Layer 1 (2 input channels) of the 9^3 feature patch (packed bf16 pairs in `in`) into the
// 7^3 patch `out`.  Chunk c's k slice of lane group g is taps l1_read_tap(c, g, q) (q = 0..3),
// one 4-byte channel pair each; the eight tap offsets of the lane are formed once per call.
template <int OUT_PLANE>
__device__ __forceinline__ void tail_layer1(const uint16_t* __restrict__ in, uint16_t* __restrict__ out,
                                            const U4 (&wr)[2], const float* __restrict__ bias) {
    constexpr int IN_E = 9, OUT_E = 7, NOUT = 343, NGRP = (NOUT + 15) / 16;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t j = lane & 15, g = lane >> 4;
    float bb[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) bb[r] = bias[4 * g + r];
    uint32_t toff[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        uint32_t tt[4];
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) {
            const int t = l1_read_tap(e >> 2, gg, e & 3);
            tt[gg] = (uint32_t)((((t / 9) * IN_E + (t / 3) % 3) * IN_E + t % 3) * 4);
        }
        toff[e] = (g & 2) ? ((g & 1) ? tt[3] : tt[2]) : ((g & 1) ? tt[1] : tt[0]);
    }
    const char* inb = reinterpret_cast<const char*>(in);
#pragma unroll 2   // two group pairs in flight: their reads overlap the other pair's products
    for (int grp = 0; grp < NGRP; grp += 2) {
        const int o0 = grp * 16 + j, o1 = o0 + 16;
        const bool v0 = o0 < NOUT, v1 = o1 < NOUT;
        const uint32_t p0 = tail_base<IN_E, OUT_E>(v0 ? o0 : NOUT - 1) * 4u;
        const uint32_t p1 = tail_base<IN_E, OUT_E>(v1 ? o1 : NOUT - 1) * 4u;
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            U4 b0, b1;
            b0.x = *reinterpret_cast<const uint32_t*>(inb + p0 + toff[4 * c + 0]);
            b0.y = *reinterpret_cast<const uint32_t*>(inb + p0 + toff[4 * c + 1]);
            b0.z = *reinterpret_cast<const uint32_t*>(inb + p0 + toff[4 * c + 2]);
            b0.w = *reinterpret_cast<const uint32_t*>(inb + p0 + toff[4 * c + 3]);
            b1.x = *reinterpret_cast<const uint32_t*>(inb + p1 + toff[4 * c + 0]);
            b1.y = *reinterpret_cast<const uint32_t*>(inb + p1 + toff[4 * c + 1]);
            b1.z = *reinterpret_cast<const uint32_t*>(inb + p1 + toff[4 * c + 2]);
            b1.w = *reinterpret_cast<const uint32_t*>(inb + p1 + toff[4 * c + 3]);
            acc0 = mfma_bf16(wr[c], b0, acc0);
            acc1 = mfma_bf16(wr[c], b1, acc1);
        }
        if (v0) tail_store<OUT_PLANE>(out, o0, g, acc0, bb);
        if (v1) tail_store<OUT_PLANE>(out, o1, g, acc1, bb);
    }
}

// The features of rounds [R0, R0 + NR) of the 9^3 patch around `node` (zero outside the
// grid), stored into Y as packed bf16 pairs.  Every lane loads a node in every round (a
// clamped in-grid node where the patch leaves the grid) and all loads are issued before
// any is used, so the rounds share one memory latency; the empty asm keeps the compiler
// from sinking each load into its own branch.
template <int R0, int NR>
__device__ __forceinline__ void tail_gather(const TailCnnArgs& a, int node, float inv_max, float inv_dd,
                                            uint16_t* Y) {
    // the lane's patch coordinates are recomputed per call (this path serves only nodes
    // near the grid's faces) rather than held in registers across the node loop
    int lane = threadIdx.x & 63;
    asm volatile("" : "+v"(lane));
    const int x0 = node % a.nx - 4, y0 = (node / a.nx) % a.ny - 4, z0 = node / (a.nx * a.ny) - 4;
    float rv[NR], ev[NR];
    uint32_t inside = 0u;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int u = lane + 64 * (R0 + r);
        const int v = u < 729 ? u : 728;
        const int x = x0 + v % 9, y = y0 + (v / 9) % 9, z = z0 + v / 81;
        const bool in = u < 729 && x >= 0 && x < a.nx && y >= 0 && y < a.ny && z >= 0 && z < a.nz;
        inside |= in ? (1u << r) : 0u;
        const int xc = min(max(x, 0), a.nx - 1), yc = min(max(y, 0), a.ny - 1), zc = min(max(z, 0), a.nz - 1);
        const int64_t n = ((int64_t)zc * a.ny + yc) * a.nx + xc;
        rv[r] = a.ref[n];
        ev[r] = a.ev[n];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        asm volatile("" : "+v"(rv[r]), "+v"(ev[r]));
        const uint32_t pk = pack2bf(rv[r] * inv_max, (ev[r] - rv[r]) * inv_dd);
        const int u = lane + 64 * (R0 + r);
        if (u < 729) reinterpret_cast<uint32_t*>(Y)[u] = ((inside >> r) & 1u) ? pk : 0u;
    }
}

// The same features for a node whose 9^3 patch lies inside the grid: voxel u of the patch
// is the patch corner plus the byte offset G[u] (G[729..767] = 0, an in-patch voxel whose
// value the masked store drops), so a round costs one table read and two loads.
template <int R0, int NR>
__device__ __forceinline__ void tail_gather_inner(const TailCnnArgs& a, int64_t corner, const uint32_t* G,
                                                  float inv_max, float inv_dd, uint16_t* Y) {
    const int lane = threadIdx.x & 63;
    const char* pr = reinterpret_cast<const char*>(a.ref + corner);
    const char* pe = reinterpret_cast<const char*>(a.ev + corner);
    float rv[NR], ev[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const uint32_t off = G[lane + 64 * (R0 + r)];
        rv[r] = *reinterpret_cast<const float*>(pr + off);
        ev[r] = *reinterpret_cast<const float*>(pe + off);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        asm volatile("" : "+v"(rv[r]), "+v"(ev[r]));
        const int u = lane + 64 * (R0 + r);
        if (64 * (R0 + r) + 63 < 729 || u < 729)
            reinterpret_cast<uint32_t*>(Y)[u] = pack2bf(rv[r] * inv_max, (ev[r] - rv[r]) * inv_dd);
    }
}

__global__ __launch_bounds__(TAIL_THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_cnn_tail(TailCnnArgs a) {
    __shared__ __align__(16) uint16_t X[TAIL_X_ELEMS];
    __shared__ __align__(16) uint16_t Y[TAIL_Y_ELEMS];
    // constants of the whole run: biases of layers 1-3, bf16-rounded layer 4 weights in
    // (tap, channel) order, layer 4 bias
    __shared__ float C[3 * 16 + 432 + 1];
    __shared__ uint32_t G[64 * TAIL_GATHER];
    const uint32_t M = *a.count;
    if (blockIdx.x >= M) return;
    const int lane = threadIdx.x & 63;
    const float inv_max = 1.0f / ord_to_float(a.sc->dmax_ord);
    const float inv_dd = a.sc->inv_dd;
    // fragments of layers 1-3, held for the whole run
    U4 w0[2], w1[14], w2[14];
#pragma unroll
    for (int c = 0; c < 2; ++c) w0[c] = reinterpret_cast<const U4*>(a.frag[0])[c * 64 + lane];
#pragma unroll
    for (int c = 0; c < 14; ++c) {
        w1[c] = reinterpret_cast<const U4*>(a.frag[1])[c * 64 + lane];
        w2[c] = reinterpret_cast<const U4*>(a.frag[2])[c * 64 + lane];
    }
    constexpr int K4 = (432 + 63) / 64;   // layer 4: 27 taps x 16 channels, tap-major
    {
        // every load issued before the first store: one memory latency for the constants
        constexpr int NC = 3 * 16 + 432 + 1, RC = (NC + 63) / 64;
        float cv[RC];
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            const int k = lane + 64 * r;
            const float* src = k < 48 ? (k < 16 ? a.bias[0] : (k < 32 ? a.bias[1] : a.bias[2])) + (k & 15)
                                      : (k < 48 + 432 ? a.w4 + ((k - 48) & 15) * 27 + ((k - 48) >> 4) : a.b4);
            cv[r] = k < NC ? *src : 0.f;
        }
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            const int k = lane + 64 * r;
            if (k < NC) C[k] = (k >= 48 && k < 48 + 432) ? bf2f(f2bf(cv[r])) : cv[r];
        }
    }
    for (int u = lane; u < 64 * TAIL_GATHER; u += 64) {
        const int v = u < 729 ? u : 0;
        G[u] = (uint32_t)((((int64_t)(v / 81) * a.ny + (v / 9) % 9) * a.nx + v % 9) * 4);
    }
    __syncthreads();
    const int64_t plane = (int64_t)a.nx * a.ny;
    const bool offs32 = plane * 9 * 4 < (int64_t(1) << 32);   // G's byte offsets fit 32 bits

    int node_next = (int)a.nodes[blockIdx.x];
    for (uint32_t item = blockIdx.x; item < M; item += gridDim.x) {
        const int node = node_next;
        if (item + gridDim.x < M) node_next = (int)a.nodes[item + gridDim.x];
        // Y is free: the previous node's layer 3 read it before the barrier that followed
        const int x = node % a.nx, y = (node / a.nx) % a.ny, z = node / (a.nx * a.ny);
        if (offs32 && x >= 4 && x + 4 < a.nx && y >= 4 && y + 4 < a.ny && z >= 4 && z + 4 < a.nz) {
            const int64_t corner = node - 4 * (plane + a.nx + 1);
            tail_gather_inner<0, TAIL_GATHER / 2>(a, corner, G, inv_max, inv_dd, Y);
            tail_gather_inner<TAIL_GATHER / 2, TAIL_GATHER - TAIL_GATHER / 2>(a, corner, G, inv_max, inv_dd, Y);
        } else {
            tail_gather<0, TAIL_GATHER / 2>(a, node, inv_max, inv_dd, Y);
            tail_gather<TAIL_GATHER / 2, TAIL_GATHER - TAIL_GATHER / 2>(a, node, inv_max, inv_dd, Y);
        }
        __syncthreads();
        tail_layer1<TAIL_XP>(Y, X, w0, C);
        __syncthreads();
        tail_layer16<7, 5, TAIL_XP, TAIL_YP>(X, Y, w1, C + 16);
        __syncthreads();
        tail_layer16<5, 3, TAIL_YP, TAIL_XP>(Y, X, w2, C + 32);
        __syncthreads();
        float s = 0.f;
#pragma unroll
        for (int r = 0; r < K4; ++r) {
            const int k = lane + 64 * r;   // tap k / 16, channel k % 16 (plane, then 8 per node)
            if (k < 432) s += C[48 + k] * bf2f(X[((k >> 3) & 1) * TAIL_XP + (k >> 4) * 8 + (k & 7)]);
        }
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) {
            const float y = C[48 + 432] + s;
            a.y[item] = y;
            if (a.key) a.key[item] = f2u(fmaxf(expf(y) - 0.01f, 0.0f));
        }
    }
}

int grid_for(int64_t n, int64_t cap) {
    int64_t b = (n + 255) / 256;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

}  // namespace

int64_t conv_blocks(const int o[3], int nvol) {
    return (int64_t)((o[2] + TX - 1) / TX) * ((o[1] + TY - 1) / TY) * ((o[0] + TZ - 1) / TZ) * nvol;
}

hipError_t launch_conv(int cin, int mode, const uint16_t* in, const int i[3], int64_t in_vstride,
                       const uint16_t* wfrag, const float* bias, int cout, const uint16_t* mask, void* out,
                       const int o[3], int64_t out_vstride, int off, int nvol, hipStream_t s) {
    ConvArgs a{};
    a.in = in;
    a.iz = i[0];
    a.iy = i[1];
    a.ix = i[2];
    a.in_vstride = in_vstride;
    a.wfrag = wfrag;
    a.bias = bias;
    a.cout = cout;
    a.mask = mask;
    a.out = out;
    a.oz = o[0];
    a.oy = o[1];
    a.ox = o[2];
    a.out_vstride = out_vstride;
    a.off = off;
    a.tiles_x = (o[2] + FX - 1) / FX;
    a.tiles_y = (o[1] + FY - 1) / FY;
    a.tiles_z = (o[0] + FZ - 1) / FZ;
    const int64_t nb = (int64_t)a.tiles_x * a.tiles_y * a.tiles_z * nvol;
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    // the kernel indexes nodes within one volume in 32 bits
    if ((int64_t)i[0] * i[1] * i[2] >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nb), block(FTHREADS);
    if (cin == 2 && mode == 0) hipLaunchKernelGGL((k_conv<2, 0>), grid, block, 0, s, a);
    else if (cin == 16 && mode == 0) hipLaunchKernelGGL((k_conv<16, 0>), grid, block, 0, s, a);
    else if (cin == 16 && mode == 1) hipLaunchKernelGGL(k_conv_last, grid, block, 0, s, a);
    else if (cin == 16 && mode == 2) hipLaunchKernelGGL((k_conv<16, 2>), grid, block, 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_conv12(const uint16_t* feat, const int f[3], int64_t feat_vstride, const uint16_t* wfrag1,
                         const float* bias1, const uint16_t* wfrag2, const float* bias2, uint16_t* out, const int o[3],
                         int64_t out_vstride, int nvol, hipStream_t s) {
    Conv12Args a{};
    a.feat = feat;
    a.fz = f[0];
    a.fy = f[1];
    a.fx = f[2];
    a.feat_vstride = feat_vstride;
    a.wfrag1 = wfrag1;
    a.bias1 = bias1;
    ConvArgs& l2 = a.l2;
    l2.wfrag = wfrag2;
    l2.bias = bias2;
    l2.cout = 16;
    l2.out = out;
    l2.oz = o[0];
    l2.oy = o[1];
    l2.ox = o[2];
    l2.out_vstride = out_vstride;
    l2.tiles_x = (o[2] + FX - 1) / FX;
    l2.tiles_y = (o[1] + FY - 1) / FY;
    l2.tiles_z = (o[0] + FZ - 1) / FZ;
    const int64_t nb = (int64_t)l2.tiles_x * l2.tiles_y * l2.tiles_z * nvol;
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7fffffff) return hipErrorInvalidValue;
    // the kernel indexes nodes within one volume in 32 bits
    if ((int64_t)f[0] * f[1] * f[2] >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_conv12, dim3((unsigned)nb), dim3(FTHREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_conv_bwdw(int cin, const uint16_t* x, const int i[3], int64_t x_vstride, const uint16_t* g,
                            const int o[3], int64_t g_vstride, int nvol, float* partial, hipStream_t s) {
    BwdWArgs a{};
    a.x = x;
    a.iz = i[0];
    a.iy = i[1];
    a.ix = i[2];
    a.x_vstride = x_vstride;
    a.g = g;
    a.oz = o[0];
    a.oy = o[1];
    a.ox = o[2];
    a.g_vstride = g_vstride;
    a.partial = partial;
    a.tiles_x = (o[2] + TX - 1) / TX;
    a.tiles_y = (o[1] + TY - 1) / TY;
    a.tiles_z = (o[0] + TZ - 1) / TZ;
    const int64_t nb = conv_blocks(o, nvol);
    if (nb <= 0) return hipSuccess;
    if (cin == 2) hipLaunchKernelGGL((k_conv_bwdw<2>), dim3((unsigned)nb), dim3(NTHREADS), 0, s, a);
    else if (cin == 16) hipLaunchKernelGGL((k_conv_bwdw<16>), dim3((unsigned)nb), dim3(NTHREADS), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const float* partial, int nblocks, int cin, int cout, float* grad, hipStream_t s) {
    const int n = cout * cin * 27 + cout;
    hipLaunchKernelGGL(k_grad_reduce, dim3((n + 255) / 256), dim3(256), 0, s, partial, nblocks, cin, cout, grad);
    return hipGetLastError();
}

hipError_t launch_loss(const float* y, const float* gamma, int64_t n, float scale, uint16_t* gout, float* loss_part,
                       int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_loss, dim3(nblocks), dim3(256), 0, s, y, gamma, n, scale, gout, loss_part);
    return hipGetLastError();
}

int loss_blocks(int64_t n) { return grid_for(n, 1024); }

hipError_t launch_adam(float* theta, float* m, float* v, const float* grad, int n, float lr, float beta1,
                       float beta2, float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, theta, m, v, grad, n, lr, beta1, beta2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t launch_pack(const float* w, int cin, int cout, int bwd, uint16_t* frag, hipStream_t s) {
    const int nch = bwd == 2 ? 2 : (bwd ? 14 : (cin == 16 ? 14 : 2));
    hipLaunchKernelGGL(k_pack, dim3(nch), dim3(64), 0, s, w, cin, cout, bwd, nch, frag);
    return hipGetLastError();
}

hipError_t launch_cnn_tail(const float* ref, const float* ev, const int n[3], const Scalars* sc,
                           const uint32_t* nodes, const uint32_t* count, int max_blocks, const uint16_t* const frag[3],
                           const float* const bias[3], const float* w4, const float* b4, float* y, uint32_t* key,
                           hipStream_t s) {
    TailCnnArgs a{};
    a.ref = ref;
    a.ev = ev;
    a.nz = n[0];
    a.ny = n[1];
    a.nx = n[2];
    a.sc = sc;
    a.nodes = nodes;
    a.count = count;
    for (int l = 0; l < 3; ++l) {
        a.frag[l] = frag[l];
        a.bias[l] = bias[l];
    }
    a.w4 = w4;
    a.b4 = b4;
    a.y = y;
    a.key = key;
    hipLaunchKernelGGL(k_cnn_tail, dim3(max_blocks > 0 ? max_blocks : 1), dim3(TAIL_THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_features(const float* ref, const float* ev, const int n[3], const Scalars* sc, uint16_t* feat,
                           hipStream_t s) {
    const int64_t total = (int64_t)(n[0] + 8) * (n[1] + 8) * (n[2] + 8);
    hipLaunchKernelGGL(k_features, dim3(grid_for(total, 4096)), dim3(256), 0, s, ref, ev, n[0], n[1], n[2], sc, feat);
    return hipGetLastError();
}

void pool2_shape(const int n[3], int c[3]) {
    for (int i = 0; i < 3; ++i) c[i] = (n[i] + 1) / 2;
}

hipError_t launch_features_pool2(const float* ref, const float* ev, const int n[3], const Scalars* sc,
                                 uint16_t* feat, hipStream_t s) {
    int c[3];
    pool2_shape(n, c);
    const int64_t total = (int64_t)(c[0] + 8) * (c[1] + 8) * (c[2] + 8);
    if (total >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_features_pool2, dim3(grid_for(total, 4096)), dim3(256), 0, s, ref, ev, n[0], n[1], n[2], sc,
                       feat);
    return hipGetLastError();
}

hipError_t launch_cnn_upsample(const float* yc, const int n[3], const uint32_t* nodes, const uint32_t* count,
                               int max_blocks, float* y, uint32_t* key, hipStream_t s) {
    hipLaunchKernelGGL(k_cnn_upsample, dim3(max_blocks > 0 ? max_blocks : 1), dim3(256), 0, s, yc, n[0], n[1], n[2],
                       nodes, count, y, key);
    return hipGetLastError();
}

}  // namespace gammax
