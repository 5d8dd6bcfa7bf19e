// Internal declarations of the learned-radius CNN kernels (k_cnn.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace gammax {

// Output tile of one convolution workgroup: 16 nodes along x (one MFMA column block) by
// 8 rows along y by 4 planes along z.
constexpr int CNN_TILE_X = 16, CNN_TILE_Y = 8, CNN_TILE_Z = 4;
// Floats per workgroup partial of bwd-weight: 27 taps x 16 x 16, then 16 bias sums.
constexpr int CNN_PARTIAL_STRIDE = 27 * 256 + 16;

// Parameter layout of the network (FP32, flat): per layer W[co][ci][dz][dy][dx], b[co].
constexpr int CNN_LAYERS = 4;
constexpr int CNN_CIN[CNN_LAYERS] = {2, 16, 16, 16};
constexpr int CNN_COUT[CNN_LAYERS] = {16, 16, 16, 1};
constexpr int CNN_OFF[CNN_LAYERS] = {0, 880, 7808, 14736};
constexpr int CNN_NPARAM = 15169;
// bf16 elements of one layer's fragment array (chunks x 64 lanes x 8)
constexpr int CNN_FRAG_ELEMS = 14 * 64 * 8;

struct ConvArgs {
    const uint16_t* in;      // channel-last bf16 (CIN channels)
    int iz, iy, ix;          // input volume shape
    int64_t in_vstride;      // bf16 elements between volumes
    const void* wfrag;       // fragments (16 bytes per lane per chunk)
    const float* bias;       // cout floats (modes 0, 1)
    int cout;
    const uint16_t* mask;    // mode 2: activation with the output's shape, 16 channels
    void* out;
    int oz, oy, ox;          // output volume shape
    int64_t out_vstride;     // elements (bf16 for 16 channels, floats for mode 1)
    int off;                 // input node = output node + tap + off (0 forward, -2 bwd-data)
    int tiles_x, tiles_y, tiles_z;
};

struct BwdWArgs {
    const uint16_t* x;       // layer input, channel-last bf16, shape = output + 2
    int iz, iy, ix;
    int64_t x_vstride;
    const uint16_t* g;       // output gradient, channel-last bf16, 16 channels
    int oz, oy, ox;
    int64_t g_vstride;
    float* partial;          // CNN_PARTIAL_STRIDE floats per workgroup
    int tiles_x, tiles_y, tiles_z;
};

int64_t conv_blocks(const int o[3], int nvol);
// mode 0: relu -> bf16; 1: linear -> FP32 channel 0 (the last layer, fragments packed by
// shifts: launch_pack bwd == 2); 2: bwd-data with ReLU mask -> bf16
hipError_t launch_conv(int cin, int mode, const uint16_t* in, const int i[3], int64_t in_vstride,
                       const uint16_t* wfrag, const float* bias, int cout, const uint16_t* mask, void* out,
                       const int o[3], int64_t out_vstride, int off, int nvol, hipStream_t s);
// Layers 1 and 2 fused: features f (2 channels) -> 16 -> 16 channels, ReLU after each, into
// out (shape o = f - 4), without storing layer 1's output.  Same values as two launch_conv
// calls (mode 0).
hipError_t launch_conv12(const uint16_t* feat, const int f[3], int64_t feat_vstride, const uint16_t* wfrag1,
                         const float* bias1, const uint16_t* wfrag2, const float* bias2, uint16_t* out, const int o[3],
                         int64_t out_vstride, int nvol, hipStream_t s);
hipError_t launch_conv_bwdw(int cin, const uint16_t* x, const int i[3], int64_t x_vstride, const uint16_t* g,
                            const int o[3], int64_t g_vstride, int nvol, float* partial, hipStream_t s);
hipError_t launch_grad_reduce(const float* partial, int nblocks, int cin, int cout, float* grad, hipStream_t s);
int loss_blocks(int64_t n);
hipError_t launch_loss(const float* y, const float* gamma, int64_t n, float scale, uint16_t* gout, float* loss_part,
                       int nblocks, hipStream_t s);
hipError_t launch_adam(float* theta, float* m, float* v, const float* grad, int n, float lr, float beta1,
                       float beta2, float eps, float c1, float c2, hipStream_t s);
// Fragments of one layer: bwd 0 forward, 1 bwd-data, 2 the last layer by shifts.
hipError_t launch_pack(const float* w, int cin, int cout, int bwd, uint16_t* frag, hipStream_t s);
// The network at the listed nodes only (their 9^3 patches): y[i] for node nodes[i], i < *count;
// key (optional) receives the bits of gamma_hat.  n: grid shape, slowest first.
hipError_t launch_cnn_tail(const float* ref, const float* ev, const int n[3], const Scalars* sc,
                           const uint32_t* nodes, const uint32_t* count, int max_blocks, const uint16_t* const frag[3],
                           const float* const bias[3], const float* w4, const float* b4, float* y, uint32_t* key,
                           hipStream_t s);
hipError_t launch_features(const float* ref, const float* ev, const int n[3], const Scalars* sc, uint16_t* feat,
                           hipStream_t s);
// Coarse grid of the 2x2x2 average pooling of an n grid: ceil(n / 2) per axis.
void pool2_shape(const int n[3], int c[3]);
// Features (as launch_features, with the fine grid's Dmax and inv_dd from sc) of the pair
// average-pooled 2x2x2 onto the coarse grid c = pool2_shape(n), padded by 4.
hipError_t launch_features_pool2(const float* ref, const float* ev, const int n[3], const Scalars* sc,
                                 uint16_t* feat, hipStream_t s);
// y at the listed fine nodes from the network output yc on the coarse grid of the pooled
// pair: gamma_hat + 0.01 = exp(yc) interpolated trilinearly, y its log; key as launch_cnn_tail.
hipError_t launch_cnn_upsample(const float* yc, const int n[3], const uint32_t* nodes, const uint32_t* count,
                               int max_blocks, float* y, uint32_t* key, hipStream_t s);

}  // namespace gammax
