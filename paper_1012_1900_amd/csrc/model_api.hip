// C ABI of the learned search radius: the model object, its forward pass over volumes,
// and one training step (forward, masked MSE on log(gamma + 0.01), backward, Adam).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gammax.h"
#include "model.hpp"

using namespace gammax;

namespace {

gammax_status_t mfail(gammax_model* m, gammax_status_t st, const std::string& why) {
    if (m) m->err = why;
    return st;
}

#define MCHK(m, call)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return mfail((m), (e_ == hipErrorOutOfMemory) ? GAMMAX_E_NOMEM : GAMMAX_E_DEVICE,       \
                         std::string(#call) + ": " + hipGetErrorString(e_));                       \
    } while (0)

hipError_t pack_all(gammax_model* m, hipStream_t s) {
    hipError_t e;
    for (int l = 0; l < CNN_LAYERS; ++l)
        if ((e = launch_pack(m->theta + CNN_OFF[l], CNN_CIN[l], CNN_COUT[l], l == 3 ? 2 : 0, frag_fwd(m, l), s)) !=
            hipSuccess)
            return e;
    for (int l = 1; l < CNN_LAYERS; ++l)
        if ((e = launch_pack(m->theta + CNN_OFF[l], CNN_CIN[l], CNN_COUT[l], 1, frag_bwd(m, l), s)) != hipSuccess)
            return e;
    return hipSuccess;
}

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

gammax_status_t check_crop(gammax_model* m, int32_t nvol, const int64_t* crop, int o[3]) {
    if (!crop) return mfail(m, GAMMAX_E_NULL, "crop shape is required");
    if (nvol < 1) return mfail(m, GAMMAX_E_PARAM, "nvol must be >= 1");
    int64_t tot = nvol;
    for (int i = 0; i < 3; ++i) {
        if (crop[i] < 1 || crop[i] > 4096) return mfail(m, GAMMAX_E_SHAPE, "crop axis must lie in [1, 4096]");
        o[i] = (int)crop[i];
        tot *= crop[i] + 8;
    }
    if (tot >= ((int64_t)1 << 31)) return mfail(m, GAMMAX_E_SHAPE, "batch too large");
    return GAMMAX_OK;
}

}  // namespace

namespace gammax {

hipError_t model_forward(gammax_model* m, const uint16_t* feat, int nvol, const int o[3], uint16_t* a1, uint16_t* a2,
                         uint16_t* a3, float* y, hipStream_t s) {
    int p0[3], s1[3], s2[3], s3[3];
    act_shape(o, 8, p0);
    act_shape(o, 6, s1);
    act_shape(o, 4, s2);
    act_shape(o, 2, s3);
    hipError_t e;
    if (!a1) {
        // layers 1 and 2 in one pass, layer 1's output kept on chip
        if ((e = launch_conv12(feat, p0, vol_of(p0) * 2, frag_fwd(m, 0), layer_bias(m, 0), frag_fwd(m, 1),
                               layer_bias(m, 1), a2, s2, vol_of(s2) * 16, nvol, s)) != hipSuccess)
            return e;
    } else {
        if ((e = launch_conv(2, 0, feat, p0, vol_of(p0) * 2, frag_fwd(m, 0), layer_bias(m, 0), 16, nullptr, a1, s1,
                             vol_of(s1) * 16, 0, nvol, s)) != hipSuccess)
            return e;
        if ((e = launch_conv(16, 0, a1, s1, vol_of(s1) * 16, frag_fwd(m, 1), layer_bias(m, 1), 16, nullptr, a2, s2,
                             vol_of(s2) * 16, 0, nvol, s)) != hipSuccess)
            return e;
    }
    if ((e = launch_conv(16, 0, a2, s2, vol_of(s2) * 16, frag_fwd(m, 2), layer_bias(m, 2), 16, nullptr, a3, s3,
                         vol_of(s3) * 16, 0, nvol, s)) != hipSuccess)
        return e;
    return launch_conv(16, 1, a3, s3, vol_of(s3) * 16, frag_fwd(m, 3), layer_bias(m, 3), 1, nullptr, y, o, vol_of(o),
                       0, nvol, s);
}

}  // namespace gammax

namespace {

// Training workspace layout for nvol volumes of output shape o.
struct TrainWs {
    uint16_t *a1, *a2, *a3, *g4, *g3, *g2, *g1;
    float *y, *partial, *loss_part;
    int64_t bytes;
    int nb_partial, nb_loss;
};

TrainWs train_layout(unsigned char* base, int nvol, const int o[3]) {
    int s1[3], s2[3], s3[3];
    act_shape(o, 6, s1);
    act_shape(o, 4, s2);
    act_shape(o, 2, s3);
    TrainWs w{};
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        unsigned char* p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    };
    w.a1 = (uint16_t*)take(nvol * vol_of(s1) * 32);
    w.a2 = (uint16_t*)take(nvol * vol_of(s2) * 32);
    w.a3 = (uint16_t*)take(nvol * vol_of(s3) * 32);
    w.y = (float*)take(nvol * vol_of(o) * 4);
    w.g4 = (uint16_t*)take(nvol * vol_of(o) * 32);
    w.g3 = (uint16_t*)take(nvol * vol_of(s3) * 32);
    w.g2 = (uint16_t*)take(nvol * vol_of(s2) * 32);
    w.g1 = (uint16_t*)take(nvol * vol_of(s1) * 32);
    w.nb_partial = (int)conv_blocks(s1, nvol);   // the largest bwd-weight grid (layer 0)
    w.partial = (float*)take((int64_t)w.nb_partial * CNN_PARTIAL_STRIDE * 4);
    w.nb_loss = loss_blocks(nvol * vol_of(o));
    w.loss_part = (float*)take((int64_t)w.nb_loss * 4);
    w.bytes = off;
    return w;
}

}  // namespace

extern "C" {

gammax_status_t gammax_model_create(int device, const float* params, gammax_model_t** out) {
    if (!out) return GAMMAX_E_NULL;
    *out = nullptr;
    if (!params) return GAMMAX_E_NULL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GAMMAX_E_DEVICE;
    for (int i = 0; i < CNN_NPARAM; ++i)
        if (!std::isfinite(params[i])) return GAMMAX_E_PARAM;
    gammax_model* m = new (std::nothrow) gammax_model();
    if (!m) return GAMMAX_E_NOMEM;
    m->device = device;
    const size_t pb = sizeof(float) * CNN_NPARAM;
    if (hipSetDevice(device) != hipSuccess || hipMalloc((void**)&m->theta, pb) != hipSuccess ||
        hipMalloc((void**)&m->adam_m, pb) != hipSuccess || hipMalloc((void**)&m->adam_v, pb) != hipSuccess ||
        hipMalloc((void**)&m->grad, pb) != hipSuccess ||
        hipMalloc((void**)&m->frag, sizeof(uint16_t) * CNN_FRAG_ELEMS * 7) != hipSuccess ||
        hipMalloc((void**)&m->d_cnt, 3 * sizeof(unsigned long long)) != hipSuccess ||
        hipHostMalloc((void**)&m->h_cnt, 3 * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
        gammax_model_destroy(m);
        return GAMMAX_E_NOMEM;
    }
    if (hipMemcpy(m->theta, params, pb, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(m->adam_m, 0, pb) != hipSuccess || hipMemset(m->adam_v, 0, pb) != hipSuccess ||
        hipMemset(m->grad, 0, pb) != hipSuccess ||
        hipMemset(m->frag, 0, sizeof(uint16_t) * CNN_FRAG_ELEMS * 7) != hipSuccess || pack_all(m, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        gammax_model_destroy(m);
        return GAMMAX_E_DEVICE;
    }
    *out = m;
    return GAMMAX_OK;
}

gammax_status_t gammax_model_destroy(gammax_model_t* m) {
    if (!m) return GAMMAX_OK;
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    void* dev[] = {m->theta, m->adam_m, m->adam_v, m->grad, m->frag, m->ws, m->d_cnt};
    for (void* p : dev)
        if (p) (void)hipFree(p);
    if (m->h_cnt) (void)hipHostFree(m->h_cnt);
    if (m->h_loss) (void)hipHostFree(m->h_loss);
    delete m;
    return GAMMAX_OK;
}

const char* gammax_model_last_error(const gammax_model_t* m) { return m ? m->err.c_str() : ""; }

gammax_status_t gammax_model_get_params(gammax_model_t* m, float* params, float* grad) {
    if (!m) return GAMMAX_E_NULL;
    if (!params && !grad) return mfail(m, GAMMAX_E_NULL, "params or grad is required");
    MCHK(m, hipSetDevice(m->device));
    MCHK(m, hipDeviceSynchronize());
    if (params) MCHK(m, hipMemcpy(params, m->theta, sizeof(float) * CNN_NPARAM, hipMemcpyDeviceToHost));
    if (grad) MCHK(m, hipMemcpy(grad, m->grad, sizeof(float) * CNN_NPARAM, hipMemcpyDeviceToHost));
    return GAMMAX_OK;
}

// Checkpoints: a one-line JSON header, then the parameters and Adam's two moment arrays as
// little-endian float32 (the host byte order of the x86-64 hosts of these GPUs).
static const char* kModelFormat = "gammax-model";
static const int kModelVersion = 1;

gammax_status_t gammax_model_save(const gammax_model_t* mc, const char* path) {
    gammax_model* m = const_cast<gammax_model*>(mc);
    if (!m) return GAMMAX_E_NULL;
    if (!path) return mfail(m, GAMMAX_E_NULL, "path is required");
    std::vector<float> buf((size_t)3 * CNN_NPARAM);
    MCHK(m, hipSetDevice(m->device));
    MCHK(m, hipDeviceSynchronize());
    MCHK(m, hipMemcpy(buf.data(), m->theta, sizeof(float) * CNN_NPARAM, hipMemcpyDeviceToHost));
    MCHK(m, hipMemcpy(buf.data() + CNN_NPARAM, m->adam_m, sizeof(float) * CNN_NPARAM, hipMemcpyDeviceToHost));
    MCHK(m, hipMemcpy(buf.data() + 2 * CNN_NPARAM, m->adam_v, sizeof(float) * CNN_NPARAM, hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    if (!f) return mfail(m, GAMMAX_E_MODEL, std::string("cannot open ") + path + " for writing");
    const int hn = std::fprintf(f,
                                "{\"format\": \"%s\", \"version\": %d, \"nparam\": %d, \"adam_step\": %lld, "
                                "\"arrays\": [\"params\", \"adam_m\", \"adam_v\"], \"dtype\": \"float32-le\"}\n",
                                kModelFormat, kModelVersion, CNN_NPARAM, (long long)m->step);
    const size_t w = std::fwrite(buf.data(), sizeof(float), buf.size(), f);
    const int cl = std::fclose(f);
    if (hn <= 0 || w != buf.size() || cl != 0) return mfail(m, GAMMAX_E_MODEL, std::string("cannot write ") + path);
    return GAMMAX_OK;
}

namespace {

// The integer after "key": in a header line (false when the key is missing).
bool header_int(const std::string& h, const char* key, long long* out) {
    const std::string k = std::string("\"") + key + "\":";
    const size_t at = h.find(k);
    if (at == std::string::npos) return false;
    return std::sscanf(h.c_str() + at + k.size(), " %lld", out) == 1;
}

}  // namespace

gammax_status_t gammax_model_load(int device, const char* path, gammax_model_t** out) {
    if (!out) return GAMMAX_E_NULL;
    *out = nullptr;
    if (!path) return GAMMAX_E_NULL;
    FILE* f = std::fopen(path, "rb");
    if (!f) return GAMMAX_E_MODEL;
    std::string head;
    for (int c; (c = std::fgetc(f)) != EOF && c != '\n';) {
        head.push_back((char)c);
        if (head.size() > 4096) break;
    }
    long long ver = 0, np = 0, step = 0;
    const bool ok_head = head.find(std::string("\"format\": \"") + kModelFormat + "\"") != std::string::npos &&
                         header_int(head, "version", &ver) && ver == kModelVersion && header_int(head, "nparam", &np) &&
                         np == CNN_NPARAM && header_int(head, "adam_step", &step) && step >= 0 &&
                         head.find("\"float32-le\"") != std::string::npos;
    std::vector<float> buf((size_t)3 * CNN_NPARAM);
    const size_t got = ok_head ? std::fread(buf.data(), sizeof(float), buf.size(), f) : 0;
    const bool at_end = ok_head && std::fgetc(f) == EOF;
    std::fclose(f);
    if (!ok_head || got != buf.size() || !at_end) return GAMMAX_E_MODEL;
    for (float v : buf)
        if (!std::isfinite(v)) return GAMMAX_E_MODEL;
    gammax_model* m = nullptr;
    gammax_status_t st = gammax_model_create(device, buf.data(), &m);
    if (st != GAMMAX_OK) return st;
    if (hipMemcpy(m->adam_m, buf.data() + CNN_NPARAM, sizeof(float) * CNN_NPARAM, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(m->adam_v, buf.data() + 2 * CNN_NPARAM, sizeof(float) * CNN_NPARAM, hipMemcpyHostToDevice) !=
            hipSuccess) {
        gammax_model_destroy(m);
        return GAMMAX_E_DEVICE;
    }
    m->step = step;
    *out = m;
    return GAMMAX_OK;
}

gammax_status_t gammax_model_forward(gammax_model_t* m, int32_t nvol, const int64_t* crop, const uint16_t* feat_dev,
                                     float* y_dev, void* stream) {
    if (!m) return GAMMAX_E_NULL;
    if (!feat_dev || !y_dev) return mfail(m, GAMMAX_E_NULL, "features and output are required");
    int o[3];
    gammax_status_t st = check_crop(m, nvol, crop, o);
    if (st != GAMMAX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    MCHK(m, hipSetDevice(m->device));
    TrainWs w = train_layout(nullptr, nvol, o);
    if (w.bytes > m->ws_cap) {
        if (m->ws) MCHK(m, hipFree(m->ws));
        m->ws = nullptr;
        m->ws_cap = 0;
        MCHK(m, hipMalloc((void**)&m->ws, (size_t)w.bytes));
        m->ws_cap = w.bytes;
    }
    w = train_layout(m->ws, nvol, o);
    MCHK(m, model_forward(m, feat_dev, nvol, o, nullptr, w.a2, w.a3, y_dev, s));
    MCHK(m, hipStreamSynchronize(s));
    return GAMMAX_OK;
}

gammax_status_t gammax_model_train_step(gammax_model_t* m, int32_t nvol, const int64_t* crop,
                                        const uint16_t* feat_dev, const float* gamma_dev,
                                        const gammax_adam_t* hp, double* loss, void* stream) {
    if (!m) return GAMMAX_E_NULL;
    if (!feat_dev || !gamma_dev || !hp) return mfail(m, GAMMAX_E_NULL, "features, labels and hyper-parameters are required");
    if (!(hp->lr >= 0.0f) || !(hp->beta1 >= 0.0f && hp->beta1 < 1.0f) || !(hp->beta2 >= 0.0f && hp->beta2 < 1.0f) ||
        !(hp->eps >= 0.0f))
        return mfail(m, GAMMAX_E_PARAM, "bad Adam hyper-parameters");
    int o[3];
    gammax_status_t st = check_crop(m, nvol, crop, o);
    if (st != GAMMAX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    MCHK(m, hipSetDevice(m->device));
    TrainWs w = train_layout(nullptr, nvol, o);
    if (w.bytes > m->ws_cap) {
        if (m->ws) MCHK(m, hipFree(m->ws));
        m->ws = nullptr;
        m->ws_cap = 0;
        MCHK(m, hipMalloc((void**)&m->ws, (size_t)w.bytes));
        m->ws_cap = w.bytes;
    }
    if (w.nb_loss > m->h_loss_cap) {
        if (m->h_loss) MCHK(m, hipHostFree(m->h_loss));
        m->h_loss = nullptr;
        m->h_loss_cap = 0;
        MCHK(m, hipHostMalloc((void**)&m->h_loss, sizeof(float) * w.nb_loss, hipHostMallocDefault));
        m->h_loss_cap = w.nb_loss;
    }
    w = train_layout(m->ws, nvol, o);
    int p0[3], s1[3], s2[3], s3[3];
    act_shape(o, 8, p0);
    act_shape(o, 6, s1);
    act_shape(o, 4, s2);
    act_shape(o, 2, s3);
    const int64_t n_out = nvol * vol_of(o);

    // forward; the count of labelled nodes (gamma >= 0) fixes the loss scale
    MCHK(m, model_forward(m, feat_dev, nvol, o, w.a1, w.a2, w.a3, w.y, s));
    MCHK(m, launch_pass_count(gamma_dev, n_out, m->d_cnt, s));
    MCHK(m, hipMemcpyAsync(m->h_cnt, m->d_cnt, 3 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    MCHK(m, hipStreamSynchronize(s));
    const unsigned long long cnt = m->h_cnt[0] > 0 ? m->h_cnt[0] : 1;
    const float scale = (float)(2.0 / (double)cnt);
    MCHK(m, launch_loss(w.y, gamma_dev, n_out, scale, w.g4, w.loss_part, w.nb_loss, s));

    // backward, layer 3 down to layer 0
    const uint16_t* xin[4] = {feat_dev, w.a1, w.a2, w.a3};
    const int* xshape[4] = {p0, s1, s2, s3};
    uint16_t* gout[4] = {w.g1, w.g2, w.g3, w.g4};   // gradient of layer l's output
    const int* gshape[4] = {s1, s2, s3, o};
    uint16_t* gin[4] = {nullptr, w.g1, w.g2, w.g3}; // gradient of layer l's input (l >= 1)
    for (int l = CNN_LAYERS - 1; l >= 0; --l) {
        const int cin = CNN_CIN[l];
        const int64_t xs = vol_of(xshape[l]) * cin, gs = vol_of(gshape[l]) * 16;
        MCHK(m, launch_conv_bwdw(cin, xin[l], xshape[l], xs, gout[l], gshape[l], gs, nvol, w.partial, s));
        const int nb = (int)conv_blocks(gshape[l], nvol);
        MCHK(m, launch_grad_reduce(w.partial, nb, cin, CNN_COUT[l], m->grad + CNN_OFF[l], s));
        if (l > 0) {
            // gradient of the input, times the ReLU derivative of the stored activation
            MCHK(m, launch_conv(16, 2, gout[l], gshape[l], gs, frag_bwd(m, l), nullptr, 16, xin[l], gin[l],
                                xshape[l], vol_of(xshape[l]) * 16, -2, nvol, s));
        }
    }

    // Adam on the FP32 master copy, then new bf16 fragments
    m->step += 1;
    const double c1 = 1.0 / (1.0 - std::pow((double)hp->beta1, (double)m->step));
    const double c2 = 1.0 / (1.0 - std::pow((double)hp->beta2, (double)m->step));
    MCHK(m, launch_adam(m->theta, m->adam_m, m->adam_v, m->grad, CNN_NPARAM, hp->lr, hp->beta1, hp->beta2, hp->eps,
                        (float)c1, (float)c2, s));
    MCHK(m, pack_all(m, s));
    MCHK(m, hipMemcpyAsync(m->h_loss, w.loss_part, sizeof(float) * w.nb_loss, hipMemcpyDeviceToHost, s));
    MCHK(m, hipStreamSynchronize(s));
    if (loss) {
        double acc = 0.0;
        for (int b = 0; b < w.nb_loss; ++b) acc += m->h_loss[b];
        *loss = acc / (double)cnt;
    }
    return GAMMAX_OK;
}

}  // extern "C"
