// C ABI of the learned coarse-to-fine corrector (include/lbmnet.h): buffer
// planning, the layer sequence of the forward and backward passes, and the
// optimizer step.  Every arithmetic step runs in the kernels of lbm_net.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_host.h"
#include "lbm_net_internal.h"
#include "lbmnet.h"

using namespace lbm_host;
namespace nd = lbmnet_dev;

namespace {

struct LayerDef {
    int cin, cout, relu, level;   // level: 0 coarse, 1 half, 2 fine
};
// The layer table of the network (order of the parameter array).
constexpr LayerDef LAYERS[LBMNET_LAYERS] = {
    {4, 16, 1, 0},  {16, 16, 1, 0}, {16, 32, 1, 1}, {32, 32, 1, 1}, {32, 32, 1, 1}, {32, 16, 1, 0},
    {32, 16, 1, 0}, {16, 16, 1, 0}, {16, 16, 1, 2}, {16, 16, 1, 2}, {16, 3, 0, 2},
};
enum { E1A, E1B, E2A, E2B, E2C, U1, D1A, D1B, F1, F2, HEAD };

inline int ceil16(int v) { return (v + 15) / 16 * 16; }
inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Packed shapes of one layer.
struct LayerGeom {
    int cin, cout_param, cout;   // cout: rounded up to a multiple of 4
    int mt, mpad, kpad;          // forward
    int mt_d, mpad_d, kpad_d;    // input gradient (flipped, transposed weights)
    int npad;                    // weight gradient columns
    int64_t off_w, off_b;        // in the parameter array
};

LayerGeom geom_of(int li, int64_t* running) {
    const LayerDef& L = LAYERS[li];
    LayerGeom g;
    g.cin = L.cin;
    g.cout_param = L.cout;
    g.cout = (L.cout + 3) / 4 * 4;
    g.mt = (g.cout + 15) / 16;
    g.mpad = 16 * g.mt;
    g.kpad = ceil16(27 * g.cin);
    g.mt_d = (g.cin + 15) / 16;
    g.mpad_d = 16 * g.mt_d;
    g.kpad_d = ceil16(27 * g.cout);
    g.npad = ceil16(27 * g.cin);
    g.off_w = *running;
    g.off_b = g.off_w + (int64_t)L.cout * 27 * L.cin;
    *running = g.off_b + L.cout;
    return g;
}

int64_t param_count() {
    int64_t p = 0;
    for (int i = 0; i < LBMNET_LAYERS; ++i) geom_of(i, &p);
    return p;
}

// Voxels per weight-gradient partial: at most 512 partials per layer.
int64_t wgrad_chunk(int64_t total) {
    int64_t c = (total + 511) / 512;
    c = (c + 15) / 16 * 16;
    return c < 256 ? 256 : c;
}

// Sizes of one layer-level grid.
struct Level {
    int n, d, h, w;
    int64_t vox() const { return (int64_t)n * d * h * w; }
};

}  // namespace

struct lbmnet {
    int n = 0, d = 0, h = 0, w = 0;
    bool train = false;
    hipStream_t stream = nullptr;
    LayerGeom lg[LBMNET_LAYERS];
    int64_t P = 0;
    Level lev[3];

    // device layout (byte offsets)
    size_t bytes = 0;
    size_t o_master = 0, o_grad = 0, o_m = 0, o_v = 0;
    size_t o_wt[LBMNET_LAYERS] = {}, o_wd[LBMNET_LAYERS] = {};
    size_t o_xin = 0, o_a16a = 0, o_cat = 0, o_upe2 = 0, o_c16b = 0, o_c16c = 0;
    size_t o_p = 0, o_h32a = 0, o_h32b = 0, o_h32c = 0;
    size_t o_upd1 = 0, o_f16a = 0, o_f16b = 0, o_r = 0, o_base = 0;
    size_t o_dr = 0, o_gpkf = 0, o_gfa = 0, o_gfb = 0;
    size_t o_gca = 0, o_gcb = 0, o_gcat = 0, o_gc32 = 0, o_gpkc = 0;
    size_t o_gha = 0, o_ghb = 0, o_gh16 = 0, o_gpkh = 0;
    size_t o_wpart = 0, o_bpart = 0, o_lpart = 0, o_stats = 0;

    char* dev = nullptr;
    bool params_set = false, weights_dirty = true, have_grad = false;
    int64_t adam_t = 0;

    template <class T>
    T* at(size_t off) const {
        return (T*)(dev + off);
    }
};

namespace {

void plan(lbmnet* net) {
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align256(b);
        return o;
    };
    const int64_t Vc = net->lev[0].vox(), Vh = net->lev[1].vox(), Vf = net->lev[2].vox();
    const size_t B = 2, F = 4;   // BF16, FP32
    net->o_master = take(F * net->P);
    for (int i = 0; i < LBMNET_LAYERS; ++i) {
        const LayerGeom& g = net->lg[i];
        net->o_wt[i] = take(B * g.mpad * g.kpad);
        if (net->train) net->o_wd[i] = take(B * g.mpad_d * g.kpad_d);
    }
    net->o_xin = take(B * Vc * 4);
    net->o_a16a = take(B * Vc * 16);
    net->o_cat = take(B * Vc * 32);
    net->o_upe2 = take(B * Vc * 32);
    net->o_c16b = take(B * Vc * 16);
    net->o_c16c = take(B * Vc * 16);
    net->o_p = take(B * Vh * 16);
    net->o_h32a = take(B * Vh * 32);
    net->o_h32b = take(B * Vh * 32);
    net->o_h32c = take(B * Vh * 32);
    net->o_upd1 = take(B * Vf * 16);
    net->o_f16a = take(B * Vf * 16);
    net->o_f16b = take(B * Vf * 16);
    net->o_r = take(F * Vf * 4);
    net->o_base = take(F * Vf * 4);
    if (net->train) {
        net->o_grad = take(F * net->P);
        net->o_m = take(F * net->P);
        net->o_v = take(F * net->P);
        net->o_dr = take(F * Vf * 4);
        net->o_gpkf = take(B * Vf * 16);
        net->o_gfa = take(F * Vf * 16);
        net->o_gfb = take(F * Vf * 16);
        net->o_gca = take(F * Vc * 16);
        net->o_gcb = take(F * Vc * 16);
        net->o_gcat = take(F * Vc * 32);
        net->o_gc32 = take(F * Vc * 32);
        net->o_gpkc = take(B * Vc * 16);
        net->o_gha = take(F * Vh * 32);
        net->o_ghb = take(F * Vh * 32);
        net->o_gh16 = take(F * Vh * 16);
        net->o_gpkh = take(B * Vh * 32);
        size_t wpart = 0;
        for (int i = 0; i < LBMNET_LAYERS; ++i) {
            const LayerGeom& g = net->lg[i];
            const int64_t tot = net->lev[LAYERS[i].level].vox();
            const int64_t chunk = wgrad_chunk(tot);
            const int64_t nchunks = (tot + chunk - 1) / chunk;
            const size_t s = F * nchunks * g.mpad * g.npad;
            if (s > wpart) wpart = s;
        }
        net->o_wpart = take(wpart);
        net->o_bpart = take(F * 64 * (size_t)nd::BIAS_PARTS);
        net->o_lpart = take(sizeof(double) * 2 * (size_t)((Vf + 255) / 256));
        net->o_stats = take(sizeof(double) * 2);
    }
    net->bytes = off;
}

bool sizes_ok(int n, int d, int h, int w) {
    return n >= 1 && d >= 2 && h >= 2 && w >= 32 && d % 2 == 0 && h % 2 == 0 && w % 32 == 0 && d <= 1024 &&
           h <= 1024 && w <= 1024 && (int64_t)n * d * h * w * 8 <= ((int64_t)1 << 31);
}

// Forward convolution of layer li: x BF16 (row ldx, channel offset cxo) -> y.
hipError_t conv_layer(lbmnet* net, int li, const uint16_t* x, int ldx, int cxo, void* y, int ldy, int cyo,
                      bool f32out) {
    const LayerGeom& g = net->lg[li];
    const Level& L = net->lev[LAYERS[li].level];
    nd::ConvArgs a;
    a.x = x;
    a.wt = net->at<uint16_t>(net->o_wt[li]);
    a.bias = net->at<float>(net->o_master) + g.off_b;
    a.y = y;
    a.n = L.n, a.d = L.d, a.h = L.h, a.w = L.w;
    a.cin = g.cin;
    a.cout = g.cout_param;
    a.kpad = g.kpad;
    a.ldx = ldx, a.cxo = cxo, a.ldy = ldy, a.cyo = cyo;
    a.relu = LAYERS[li].relu;
    return nd::conv_forward(a, g.mt, f32out, net->stream);
}

// Backward of layer li.  g: FP32 gradient with respect to the layer output
// (row ldg, channel offset offg), masked by the ReLU of act (g is only read;
// the masked values go to the packed BF16 copy).  x: the
// layer input.  dx: FP32 gradient with respect to the input (null: skipped).
hipError_t backward_layer(lbmnet* net, int li, float* g, int ldg, int offg, const uint16_t* act, int lda, int offa,
                          const uint16_t* x, int ldx, int cxo, uint16_t* packed, float* dx, int lddx) {
    const LayerGeom& G = net->lg[li];
    const Level& L = net->lev[LAYERS[li].level];
    const int64_t tot = L.vox();
    float* grad = net->at<float>(net->o_grad);
    nd::BiasJob bias;
    hipError_t e = nd::grad_relu_cast(g, ldg, offg, LAYERS[li].relu ? act : nullptr, lda, offa, G.cout, tot, packed,
                                      net->at<float>(net->o_bpart), G.cout_param, grad + G.off_b, net->stream, &bias);
    if (e != hipSuccess) return e;
    // weight gradient
    nd::WgradArgs w;
    w.dy = packed;
    w.x = x;
    w.part = net->at<float>(net->o_wpart);
    w.n = L.n, w.d = L.d, w.h = L.h, w.w = L.w;
    w.cin = G.cin;
    w.cout = G.cout;
    w.mpad = G.mpad;
    w.npad = G.npad;
    w.ldy = G.cout;
    w.ldx = ldx;
    w.cxo = cxo;
    w.chunk = wgrad_chunk(tot);
    const int nchunks = (int)((tot + w.chunk - 1) / w.chunk);
    e = nd::conv_wgrad(w, G.mt, nchunks, G.cout_param, grad + G.off_w, net->stream, &bias);
    if (e != hipSuccess) return e;
    if (!dx) return hipSuccess;
    // input gradient: the forward kernel with the flipped, transposed weights
    nd::ConvArgs a;
    a.x = packed;
    a.wt = net->at<uint16_t>(net->o_wd[li]);
    a.bias = nullptr;
    a.y = dx;
    a.n = L.n, a.d = L.d, a.h = L.h, a.w = L.w;
    a.cin = G.cout;
    a.cout = G.cin;
    a.kpad = G.kpad_d;
    a.ldx = G.cout, a.cxo = 0, a.ldy = lddx, a.cyo = 0;
    a.relu = 0;
    return nd::conv_forward(a, G.mt_d, true, net->stream);
}

int prepare_weights(lbmnet* net) {
    if (!net->weights_dirty) return LBM_OK;
    const float* master = net->at<float>(net->o_master);
    static_assert(LBMNET_LAYERS <= nd::MAX_PREP_JOBS, "one packing launch covers every layer");
    nd::PrepJobs jobs{};
    jobs.n = LBMNET_LAYERS;
    for (int i = 0; i < LBMNET_LAYERS; ++i) {
        const LayerGeom& g = net->lg[i];
        jobs.j[i] = nd::PrepJob{master + g.off_w, net->at<uint16_t>(net->o_wt[i]),
                                net->train ? net->at<uint16_t>(net->o_wd[i]) : nullptr, g.cin, g.cout_param, g.cout,
                                g.mpad, g.kpad, g.mpad_d, g.kpad_d};
    }
    HIP_TRY(nd::prep_weights_all(jobs, net->stream), "lbmnet weight packing");
    net->weights_dirty = false;
    return LBM_OK;
}

int run_forward(lbmnet* net, const float* x) {
    int rc = prepare_weights(net);
    if (rc != LBM_OK) return rc;
    const Level& C = net->lev[0];
    const Level& H = net->lev[1];
    auto B = [&](size_t o) { return net->at<uint16_t>(o); };
    HIP_TRY(nd::cast_input(x, C.vox() * 4, B(net->o_xin), net->stream), "lbmnet input cast");
    HIP_TRY(conv_layer(net, E1A, B(net->o_xin), 4, 0, B(net->o_a16a), 16, 0, false), "lbmnet conv e1a");
    HIP_TRY(conv_layer(net, E1B, B(net->o_a16a), 16, 0, B(net->o_cat), 32, 0, false), "lbmnet conv e1b");
    HIP_TRY(nd::avgpool_fwd(B(net->o_cat), 32, 0, 16, C.n, C.d, C.h, C.w, B(net->o_p), net->stream), "lbmnet pool");
    HIP_TRY(conv_layer(net, E2A, B(net->o_p), 16, 0, B(net->o_h32a), 32, 0, false), "lbmnet conv e2a");
    HIP_TRY(conv_layer(net, E2B, B(net->o_h32a), 32, 0, B(net->o_h32b), 32, 0, false), "lbmnet conv e2b");
    HIP_TRY(conv_layer(net, E2C, B(net->o_h32b), 32, 0, B(net->o_h32c), 32, 0, false), "lbmnet conv e2c");
    HIP_TRY(nd::upsample_fwd(B(net->o_h32c), 32, H.n, H.d, H.h, H.w, B(net->o_upe2), net->stream), "lbmnet up");
    HIP_TRY(conv_layer(net, U1, B(net->o_upe2), 32, 0, B(net->o_cat), 32, 16, false), "lbmnet conv u1");
    HIP_TRY(conv_layer(net, D1A, B(net->o_cat), 32, 0, B(net->o_c16b), 16, 0, false), "lbmnet conv d1a");
    HIP_TRY(conv_layer(net, D1B, B(net->o_c16b), 16, 0, B(net->o_c16c), 16, 0, false), "lbmnet conv d1b");
    HIP_TRY(nd::upsample_fwd(B(net->o_c16c), 16, C.n, C.d, C.h, C.w, B(net->o_upd1), net->stream), "lbmnet up");
    HIP_TRY(conv_layer(net, F1, B(net->o_upd1), 16, 0, B(net->o_f16a), 16, 0, false), "lbmnet conv f1");
    HIP_TRY(conv_layer(net, F2, B(net->o_f16a), 16, 0, B(net->o_f16b), 16, 0, false), "lbmnet conv f2");
    HIP_TRY(conv_layer(net, HEAD, B(net->o_f16b), 16, 0, net->at<float>(net->o_r), 4, 0, true), "lbmnet conv head");
    HIP_TRY(nd::trilinear(x, C.n, C.d, C.h, C.w, net->at<float>(net->o_base), 4, net->stream), "lbmnet trilinear");
    return LBM_OK;
}

int run_backward(lbmnet* net) {
    const Level& C = net->lev[0];
    const Level& H = net->lev[1];
    auto B = [&](size_t o) { return net->at<uint16_t>(o); };
    auto Fp = [&](size_t o) { return net->at<float>(o); };
    // fine level
    HIP_TRY(backward_layer(net, HEAD, Fp(net->o_dr), 4, 0, nullptr, 0, 0, B(net->o_f16b), 16, 0, B(net->o_gpkf),
                           Fp(net->o_gfa), 16),
            "lbmnet backward head");
    HIP_TRY(backward_layer(net, F2, Fp(net->o_gfa), 16, 0, B(net->o_f16b), 16, 0, B(net->o_f16a), 16, 0,
                           B(net->o_gpkf), Fp(net->o_gfb), 16),
            "lbmnet backward f2");
    HIP_TRY(backward_layer(net, F1, Fp(net->o_gfb), 16, 0, B(net->o_f16a), 16, 0, B(net->o_upd1), 16, 0,
                           B(net->o_gpkf), Fp(net->o_gfa), 16),
            "lbmnet backward f1");
    HIP_TRY(nd::upsample_bwd(Fp(net->o_gfa), 16, C.n, C.d, C.h, C.w, Fp(net->o_gca), net->stream),
            "lbmnet upsample backward");
    // coarse decoder
    HIP_TRY(backward_layer(net, D1B, Fp(net->o_gca), 16, 0, B(net->o_c16c), 16, 0, B(net->o_c16b), 16, 0,
                           B(net->o_gpkc), Fp(net->o_gcb), 16),
            "lbmnet backward d1b");
    HIP_TRY(backward_layer(net, D1A, Fp(net->o_gcb), 16, 0, B(net->o_c16b), 16, 0, B(net->o_cat), 32, 0,
                           B(net->o_gpkc), Fp(net->o_gcat), 32),
            "lbmnet backward d1a");
    HIP_TRY(backward_layer(net, U1, Fp(net->o_gcat), 32, 16, B(net->o_cat), 32, 16, B(net->o_upe2), 32, 0,
                           B(net->o_gpkc), Fp(net->o_gc32), 32),
            "lbmnet backward u1");
    HIP_TRY(nd::upsample_bwd(Fp(net->o_gc32), 32, H.n, H.d, H.h, H.w, Fp(net->o_gha), net->stream),
            "lbmnet upsample backward");
    // half level
    HIP_TRY(backward_layer(net, E2C, Fp(net->o_gha), 32, 0, B(net->o_h32c), 32, 0, B(net->o_h32b), 32, 0,
                           B(net->o_gpkh), Fp(net->o_ghb), 32),
            "lbmnet backward e2c");
    HIP_TRY(backward_layer(net, E2B, Fp(net->o_ghb), 32, 0, B(net->o_h32b), 32, 0, B(net->o_h32a), 32, 0,
                           B(net->o_gpkh), Fp(net->o_gha), 32),
            "lbmnet backward e2b");
    HIP_TRY(backward_layer(net, E2A, Fp(net->o_gha), 32, 0, B(net->o_h32a), 32, 0, B(net->o_p), 16, 0,
                           B(net->o_gpkh), Fp(net->o_gh16), 16),
            "lbmnet backward e2a");
    // skip connection: the pooled branch adds into the e1 part of the concat gradient
    HIP_TRY(nd::avgpool_bwd_add(Fp(net->o_gh16), 16, C.n, C.d, C.h, C.w, Fp(net->o_gcat), 32, 0, net->stream),
            "lbmnet pool backward");
    HIP_TRY(backward_layer(net, E1B, Fp(net->o_gcat), 32, 0, B(net->o_cat), 32, 0, B(net->o_a16a), 16, 0,
                           B(net->o_gpkc), Fp(net->o_gca), 16),
            "lbmnet backward e1b");
    HIP_TRY(backward_layer(net, E1A, Fp(net->o_gca), 16, 0, B(net->o_a16a), 16, 0, B(net->o_xin), 4, 0,
                           B(net->o_gpkc), nullptr, 0),
            "lbmnet backward e1a");
    return LBM_OK;
}

int check_net(const lbmnet* net, const char* what) {
    if (!net) return fail(LBM_EINVAL, std::string(what) + ": null network");
    if (!net->dev) return fail(LBM_ESTATE, std::string(what) + ": no device memory attached");
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbmnet_param_count(int64_t* n) {
    if (!n) return fail(LBM_EINVAL, "lbmnet_param_count: null output");
    *n = param_count();
    return LBM_OK;
}

int lbmnet_layer_info(int i, int64_t info[5]) {
    if (!info || i < 0 || i >= LBMNET_LAYERS) return fail(LBM_EINVAL, "lbmnet_layer_info: bad layer index");
    int64_t p = 0;
    LayerGeom g{};
    for (int k = 0; k <= i; ++k) g = geom_of(k, &p);
    info[0] = LAYERS[i].cin;
    info[1] = LAYERS[i].cout;
    info[2] = LAYERS[i].relu;
    info[3] = LAYERS[i].level;
    info[4] = g.off_w;
    return LBM_OK;
}

int lbmnet_create(int n, int d, int h, int w, int train, void* hip_stream, lbmnet** out) {
    if (!out) return fail(LBM_EINVAL, "lbmnet_create: null output");
    *out = nullptr;
    if (!sizes_ok(n, d, h, w))
        return fail(LBM_EINVAL, "lbmnet_create: need n >= 1, even d and h, w a multiple of 32, sizes <= 1024");
    lbmnet* net = new (std::nothrow) lbmnet();
    if (!net) return fail(LBM_ENOMEM, "lbmnet_create: out of host memory");
    net->n = n, net->d = d, net->h = h, net->w = w;
    net->train = train != 0;
    net->stream = (hipStream_t)hip_stream;
    int64_t p = 0;
    for (int i = 0; i < LBMNET_LAYERS; ++i) net->lg[i] = geom_of(i, &p);
    net->P = p;
    net->lev[0] = Level{n, d, h, w};
    net->lev[1] = Level{n, d / 2, h / 2, w / 2};
    net->lev[2] = Level{n, 2 * d, 2 * h, 2 * w};
    plan(net);
    *out = net;
    return LBM_OK;
}

int lbmnet_device_bytes(const lbmnet* net, size_t* bytes) {
    if (!net || !bytes) return fail(LBM_EINVAL, "lbmnet_device_bytes: null argument");
    *bytes = net->bytes;
    return LBM_OK;
}

int lbmnet_attach_device(lbmnet* net, void* dev_ptr, size_t bytes) {
    if (!net || !dev_ptr) return fail(LBM_EINVAL, "lbmnet_attach_device: null argument");
    if (((uintptr_t)dev_ptr) % 256 != 0) return fail(LBM_EINVAL, "lbmnet_attach_device: pointer not 256-byte aligned");
    if (bytes < net->bytes) return fail(LBM_ENOMEM, "lbmnet_attach_device: buffer too small");
    net->dev = (char*)dev_ptr;
    // the head writes 3 of the 4 channels of r; keep the fourth defined
    HIP_TRY(nd::fill(net->at<float>(net->o_r), sizeof(float) * 4 * net->lev[2].vox(), 0u, net->stream),
            "lbmnet attach");
    net->params_set = false;
    net->have_grad = false;
    return LBM_OK;
}

int lbmnet_set_params(lbmnet* net, const float* params) {
    int rc = check_net(net, "lbmnet_set_params");
    if (rc != LBM_OK) return rc;
    if (!params) return fail(LBM_EINVAL, "lbmnet_set_params: null parameters");
    for (int64_t i = 0; i < net->P; ++i)
        if (!std::isfinite(params[i])) return fail(LBM_EINVAL, "lbmnet_set_params: non-finite parameter");
    HIP_TRY(hipMemcpyAsync(net->at<float>(net->o_master), params, sizeof(float) * net->P, hipMemcpyHostToDevice,
                           net->stream),
            "lbmnet_set_params copy");
    if (net->train) {
        HIP_TRY(nd::fill(net->at<float>(net->o_m), sizeof(float) * net->P, 0u, net->stream), "lbmnet_set_params");
        HIP_TRY(nd::fill(net->at<float>(net->o_v), sizeof(float) * net->P, 0u, net->stream), "lbmnet_set_params");
    }
    HIP_TRY(hipStreamSynchronize(net->stream), "lbmnet_set_params sync");
    net->adam_t = 0;
    net->params_set = true;
    net->weights_dirty = true;
    net->have_grad = false;
    return LBM_OK;
}

int lbmnet_get_params(lbmnet* net, float* params) {
    int rc = check_net(net, "lbmnet_get_params");
    if (rc != LBM_OK) return rc;
    if (!params) return fail(LBM_EINVAL, "lbmnet_get_params: null output");
    if (!net->params_set) return fail(LBM_ESTATE, "lbmnet_get_params: parameters not set");
    HIP_TRY(hipMemcpyAsync(params, net->at<float>(net->o_master), sizeof(float) * net->P, hipMemcpyDeviceToHost,
                           net->stream),
            "lbmnet_get_params copy");
    HIP_TRY(hipStreamSynchronize(net->stream), "lbmnet_get_params sync");
    return LBM_OK;
}

int lbmnet_forward(lbmnet* net, const float* x, float* out) {
    int rc = check_net(net, "lbmnet_forward");
    if (rc != LBM_OK) return rc;
    if (!x || !out) return fail(LBM_EINVAL, "lbmnet_forward: null tensor");
    if (!net->params_set) return fail(LBM_ESTATE, "lbmnet_forward: parameters not set");
    rc = run_forward(net, x);
    if (rc != LBM_OK) return rc;
    HIP_TRY(nd::add_residual(net->at<float>(net->o_base), net->at<float>(net->o_r), net->lev[2].vox(), out,
                             net->stream),
            "lbmnet output");
    return LBM_OK;
}

int lbmnet_loss_grad(lbmnet* net, const float* x, const float* target, const uint8_t* mask, double* loss,
                     float* grad) {
    int rc = check_net(net, "lbmnet_loss_grad");
    if (rc != LBM_OK) return rc;
    if (!x || !target || !mask) return fail(LBM_EINVAL, "lbmnet_loss_grad: null tensor");
    if (!net->train) return fail(LBM_ESTATE, "lbmnet_loss_grad: network created without training buffers");
    if (!net->params_set) return fail(LBM_ESTATE, "lbmnet_loss_grad: parameters not set");
    rc = run_forward(net, x);
    if (rc != LBM_OK) return rc;
    HIP_TRY(nd::loss_and_grad(net->at<float>(net->o_base), net->at<float>(net->o_r), target, mask, net->lev[2].vox(),
                              net->at<double>(net->o_lpart), net->at<double>(net->o_stats),
                              net->at<float>(net->o_dr), net->stream),
            "lbmnet loss");
    rc = run_backward(net);
    if (rc != LBM_OK) return rc;
    net->have_grad = true;
    if (grad)
        HIP_TRY(hipMemcpyAsync(grad, net->at<float>(net->o_grad), sizeof(float) * net->P, hipMemcpyDeviceToDevice,
                               net->stream),
                "lbmnet gradient copy");
    if (loss) {
        double st[2];
        HIP_TRY(hipMemcpyAsync(st, net->at<double>(net->o_stats), sizeof(st), hipMemcpyDeviceToHost, net->stream),
                "lbmnet loss copy");
        HIP_TRY(hipStreamSynchronize(net->stream), "lbmnet loss sync");
        *loss = st[0];
        if (!std::isfinite(st[0])) return fail(LBM_EUNSTABLE, "lbmnet_loss_grad: non-finite loss");
    }
    return LBM_OK;
}

int lbmnet_adam_step(lbmnet* net, float lr, float b1, float b2, float eps) {
    int rc = check_net(net, "lbmnet_adam_step");
    if (rc != LBM_OK) return rc;
    if (!(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps >= 0) || !std::isfinite(lr))
        return fail(LBM_EINVAL, "lbmnet_adam_step: need lr > 0, 0 <= b1, b2 < 1, eps >= 0");
    if (!net->train || !net->have_grad) return fail(LBM_ESTATE, "lbmnet_adam_step: no gradient");
    net->adam_t += 1;
    const double c1 = 1.0 - std::pow((double)b1, (double)net->adam_t);
    const double c2 = 1.0 - std::pow((double)b2, (double)net->adam_t);
    HIP_TRY(nd::adam(net->at<float>(net->o_master), net->at<float>(net->o_grad), net->at<float>(net->o_m),
                     net->at<float>(net->o_v), net->P, lr, b1, b2, eps, (float)c1, (float)c2, net->stream),
            "lbmnet adam");
    net->weights_dirty = true;
    return LBM_OK;
}

int lbmnet_adam_count(const lbmnet* net, int64_t* t) {
    if (!net || !t) return fail(LBM_EINVAL, "lbmnet_adam_count: null argument");
    *t = net->adam_t;
    return LBM_OK;
}

int lbmnet_destroy(lbmnet* net) {
    delete net;
    return LBM_OK;
}

// ---- one convolution layer ------------------------------------------------------

namespace {
struct ConvWork {
    size_t xb, yb, wt, wd, gb, wpart, bpart, total;
};
bool conv_sizes_ok(int n, int d, int h, int w, int cin, int cout) {
    return n >= 1 && d >= 1 && h >= 1 && w >= 16 && w % 16 == 0 && cin >= 4 && cin <= 32 && cin % 4 == 0 &&
           (cout == 4 || cout == 8 || cout == 16 || cout == 32) && (int64_t)n * d * h * w * 32 < ((int64_t)1 << 31);
}
ConvWork conv_work(int n, int d, int h, int w, int cin, int cout) {
    const int64_t V = (int64_t)n * d * h * w;
    const int mpad = ceil16(cout), kpad = ceil16(27 * cin), mpad_d = ceil16(cin), kpad_d = ceil16(27 * cout);
    const int64_t chunk = wgrad_chunk(V);
    const int64_t nchunks = (V + chunk - 1) / chunk;
    ConvWork c;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off += align256(b);
        return o;
    };
    c.xb = take(2 * V * cin);
    c.yb = take(2 * V * cout);
    c.wt = take(2 * (size_t)mpad * kpad);
    c.wd = take(2 * (size_t)mpad_d * kpad_d);
    c.gb = take(2 * V * cout);
    c.wpart = take(4 * (size_t)nchunks * mpad * ceil16(27 * cin));
    c.bpart = take(4 * 64 * (size_t)nd::BIAS_PARTS);
    c.total = off;
    return c;
}
}  // namespace

int lbmnet_conv3d_workspace(int n, int d, int h, int w, int cin, int cout, size_t* bytes) {
    if (!bytes) return fail(LBM_EINVAL, "lbmnet_conv3d_workspace: null output");
    if (!conv_sizes_ok(n, d, h, w, cin, cout)) return fail(LBM_EINVAL, "lbmnet_conv3d_workspace: bad sizes");
    *bytes = conv_work(n, d, h, w, cin, cout).total;
    return LBM_OK;
}

int lbmnet_conv3d(int n, int d, int h, int w, int cin, int cout, int relu, const float* x, const float* wts,
                  const float* b, const float* dy, float* y, float* dx, float* dw, float* db, void* work,
                  size_t work_bytes, void* hip_stream) {
    if (!conv_sizes_ok(n, d, h, w, cin, cout)) return fail(LBM_EINVAL, "lbmnet_conv3d: bad sizes");
    if (!x || !wts || !b || !y || !work) return fail(LBM_EINVAL, "lbmnet_conv3d: null tensor");
    if (dy && (!dx || !dw || !db)) return fail(LBM_EINVAL, "lbmnet_conv3d: backward needs dx, dw and db");
    if (((uintptr_t)work) % 256 != 0) return fail(LBM_EINVAL, "lbmnet_conv3d: workspace not 256-byte aligned");
    const ConvWork cw = conv_work(n, d, h, w, cin, cout);
    if (work_bytes < cw.total) return fail(LBM_ENOMEM, "lbmnet_conv3d: workspace too small");
    hipStream_t st = (hipStream_t)hip_stream;
    char* base = (char*)work;
    const int64_t V = (int64_t)n * d * h * w;
    const int mt = (cout + 15) / 16, mpad = 16 * mt, kpad = ceil16(27 * cin);
    const int mt_d = (cin + 15) / 16, mpad_d = 16 * mt_d, kpad_d = ceil16(27 * cout);
    uint16_t* xb = (uint16_t*)(base + cw.xb);
    uint16_t* yb = (uint16_t*)(base + cw.yb);
    uint16_t* wt = (uint16_t*)(base + cw.wt);
    uint16_t* wd = (uint16_t*)(base + cw.wd);
    uint16_t* gb = (uint16_t*)(base + cw.gb);
    HIP_TRY(nd::cast_input(x, V * cin, xb, st), "lbmnet_conv3d cast");
    HIP_TRY(nd::prep_weights(wts, cin, cout, cout, wt, mpad, kpad, wd, mpad_d, kpad_d, st), "lbmnet_conv3d weights");
    nd::ConvArgs a;
    a.x = xb;
    a.wt = wt;
    a.bias = b;
    a.y = y;
    a.n = n, a.d = d, a.h = h, a.w = w;
    a.cin = cin, a.cout = cout, a.kpad = kpad;
    a.ldx = cin, a.cxo = 0, a.ldy = cout, a.cyo = 0;
    a.relu = relu ? 1 : 0;
    HIP_TRY(nd::conv_forward(a, mt, true, st), "lbmnet_conv3d forward");
    if (!dy) return LBM_OK;
    a.y = yb;
    HIP_TRY(nd::conv_forward(a, mt, false, st), "lbmnet_conv3d forward (BF16 copy)");
    HIP_TRY(nd::grad_relu_cast(dy, cout, 0, relu ? yb : nullptr, cout, 0, cout, V, gb, (float*)(base + cw.bpart), cout,
                               db, st),
            "lbmnet_conv3d mask and bias gradient");
    nd::WgradArgs wa;
    wa.dy = gb;
    wa.x = xb;
    wa.part = (float*)(base + cw.wpart);
    wa.n = n, wa.d = d, wa.h = h, wa.w = w;
    wa.cin = cin, wa.cout = cout, wa.mpad = mpad, wa.npad = ceil16(27 * cin);
    wa.ldy = cout, wa.ldx = cin, wa.cxo = 0;
    wa.chunk = wgrad_chunk(V);
    const int nchunks = (int)((V + wa.chunk - 1) / wa.chunk);
    HIP_TRY(nd::conv_wgrad(wa, mt, nchunks, cout, dw, st), "lbmnet_conv3d weight gradient");
    nd::ConvArgs t;
    t.x = gb;
    t.wt = wd;
    t.bias = nullptr;
    t.y = dx;
    t.n = n, t.d = d, t.h = h, t.w = w;
    t.cin = cout, t.cout = cin, t.kpad = kpad_d;
    t.ldx = cout, t.cxo = 0, t.ldy = cin, t.cyo = 0;
    t.relu = 0;
    HIP_TRY(nd::conv_forward(t, mt_d, true, st), "lbmnet_conv3d input gradient");
    return LBM_OK;
}

// ---- data movement ----------------------------------------------------------------

int lbmnet_scatter(const double* vals, const int32_t* xyz, int64_t count, int D, int H, int W, double scale,
                   float* dense, uint8_t* mask, void* hip_stream) {
    if ((!vals || !xyz) && count > 0) return fail(LBM_EINVAL, "lbmnet_scatter: null node arrays");
    if (!dense || !mask || D < 1 || H < 1 || W < 1 || count < 0 || !std::isfinite(scale))
        return fail(LBM_EINVAL, "lbmnet_scatter: bad grid or scale");
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t V = (size_t)D * H * W;
    HIP_TRY(nd::fill(dense, sizeof(float) * 3 * V, 0u, st), "lbmnet_scatter clear");
    HIP_TRY(nd::fill(mask, V / 4 * 4, 0u, st), "lbmnet_scatter clear");
    if (V % 4) HIP_TRY(hipMemsetAsync(mask + V / 4 * 4, 0, V % 4, st), "lbmnet_scatter clear");
    if (count == 0) return LBM_OK;
    HIP_TRY(nd::scatter(vals, xyz, count, D, H, W, scale, dense, mask, st), "lbmnet_scatter");
    return LBM_OK;
}

int lbmnet_gather(const float* dense, const int32_t* xyz, int64_t count, int D, int H, int W, double scale,
                  double* vals, void* hip_stream) {
    if (count < 0 || D < 1 || H < 1 || W < 1 || !dense || !std::isfinite(scale))
        return fail(LBM_EINVAL, "lbmnet_gather: bad grid or scale");
    if (count == 0) return LBM_OK;
    if (!vals || !xyz) return fail(LBM_EINVAL, "lbmnet_gather: null node arrays");
    HIP_TRY(nd::gather(dense, xyz, count, D, H, W, scale, vals, (hipStream_t)hip_stream), "lbmnet_gather");
    return LBM_OK;
}

int lbmnet_crop(const float* uc, const uint8_t* mc, int Dc, int Hc, int Wc, const float* uf, const uint8_t* mf,
                const int32_t* origins, int n, int d, int h, int w, int margin, float* xin, float* target,
                uint8_t* tmask, void* hip_stream) {
    if (!uc || !mc || !uf || !mf || !origins || !xin || !target || !tmask)
        return fail(LBM_EINVAL, "lbmnet_crop: null tensor");
    if (Dc < 1 || Hc < 1 || Wc < 1 || n < 1 || d < 1 || h < 1 || w < 1 || margin < 0 ||
        (int64_t)n * d * h * w * 8 > ((int64_t)1 << 31))
        return fail(LBM_EINVAL, "lbmnet_crop: bad sizes");
    HIP_TRY(nd::crop(uc, mc, Dc, Hc, Wc, uf, mf, origins, n, d, h, w, margin, xin, target, tmask,
                     (hipStream_t)hip_stream),
            "lbmnet_crop");
    return LBM_OK;
}

int lbmnet_trilinear(const float* x, int n, int d, int h, int w, float* out, void* hip_stream) {
    if (!x || !out || n < 1 || d < 1 || h < 1 || w < 1 || (int64_t)n * d * h * w * 8 > ((int64_t)1 << 31))
        return fail(LBM_EINVAL, "lbmnet_trilinear: bad arguments");
    HIP_TRY(nd::trilinear(x, n, d, h, w, out, 3, (hipStream_t)hip_stream), "lbmnet_trilinear");
    return LBM_OK;
}

}  // extern "C"
