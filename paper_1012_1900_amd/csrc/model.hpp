// The learned-radius model object shared by the C ABI translation units.
#pragma once

#include <string>

#include "cnn.hpp"

struct gammax_model {
    int device = 0;
    std::string err;
    float* theta = nullptr;     // FP32 master parameters, CNN_NPARAM (flat layout of the header)
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    float* grad = nullptr;      // gradient of the last training step
    uint16_t* frag = nullptr;   // bf16 fragments: forward layers 0..3, then bwd-data layers 1..3
    int64_t step = 0;           // Adam steps taken
    // training workspace (grown on demand)
    unsigned char* ws = nullptr;
    int64_t ws_cap = 0;
    unsigned long long* d_cnt = nullptr;
    unsigned long long* h_cnt = nullptr;   // pinned
    float* h_loss = nullptr;               // pinned, loss partials
    int64_t h_loss_cap = 0;
};

namespace gammax {

inline uint16_t* frag_fwd(gammax_model* m, int l) { return m->frag + (int64_t)l * CNN_FRAG_ELEMS; }
inline uint16_t* frag_bwd(gammax_model* m, int l) { return m->frag + (int64_t)(3 + l) * CNN_FRAG_ELEMS; }
inline const float* layer_bias(const gammax_model* m, int l) {
    return m->theta + CNN_OFF[l] + CNN_COUT[l] * CNN_CIN[l] * 27;
}

// Shapes of the activations for an output (grid or crop) shape o: features o + 8,
// layer outputs o + 6, o + 4, o + 2, then o.
inline void act_shape(const int o[3], int grow, int out[3]) {
    for (int i = 0; i < 3; ++i) out[i] = o[i] + grow;
}
inline int64_t vol_of(const int s[3]) { return (int64_t)s[0] * s[1] * s[2]; }

// Forward pass over nvol volumes: feat (o+8, 2 channels) -> a1 (o+6), a2 (o+4),
// a3 (o+2) (16 channels each, bf16) -> y (o, FP32).  a1 == nullptr: layers 1 and 2 run
// fused and a1 is not stored (inference; training keeps it for the backward pass).
hipError_t model_forward(gammax_model* m, const uint16_t* feat, int nvol, const int o[3], uint16_t* a1, uint16_t* a2,
                         uint16_t* a3, float* y, hipStream_t s);

}  // namespace gammax
