// Kernel arguments and launchers of the learned corrector (lbm_net.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lbmnet_dev {

constexpr int BIAS_PARTS = 1024;   // work-groups of the bias-gradient sums

// 3x3x3 convolution as an implicit GEMM.  x: BF16 channels [cxo, cxo + cin)
// of rows of length ldx; wt: BF16 [mpad][kpad], K = 27 cin tap-major (zero
// padded); y: rows of length ldy, channels [cyo, cyo + cout), FP32 or BF16.
// Requirements: w % 16 == 0, cin % 4 == 0, cout <= 16 * MT.
struct ConvArgs {
    const uint16_t* x;
    const uint16_t* wt;
    const float* bias;   // may be null
    void* y;
    int n, d, h, w;
    int cin, cout, kpad;
    int ldx, cxo, ldy, cyo;
    int relu;
};

// Weight gradient: dy BF16 [V][ldy] (channels 0..cout), x as in ConvArgs;
// part: FP32 [nchunks][mpad][npad], npad = 16 * ceil(27 cin / 16).
struct WgradArgs {
    const uint16_t* dy;
    const uint16_t* x;
    float* part;
    int n, d, h, w;
    int cin, cout, mpad, npad;
    int ldy, ldx, cxo;
    int64_t chunk;   // voxels per partial, multiple of 16
};

// Bias-gradient partials waiting for their reduction: part [nparts][64],
// channels < cout_param summed into db.
struct BiasJob {
    const float* part;
    int nparts, cout_param;
    float* db;
};

// FP32 master weights of one layer packed to the BF16 forward (wt) and
// input-gradient (wd, may be null) matrices; see prep_weights.
struct PrepJob {
    const float* w;
    uint16_t* wt;
    uint16_t* wd;
    int cin, cout_param, cout, mpad, kpad, mpad_d, kpad_d;
};
constexpr int MAX_PREP_JOBS = 16;
struct PrepJobs {
    PrepJob j[MAX_PREP_JOBS];
    int n;
};

hipError_t conv_forward(const ConvArgs& a, int mt, bool f32out, hipStream_t st);
// bias (may be null): a deferred bias-gradient reduction, done in the same
// launch as the weight-gradient reduction.
hipError_t conv_wgrad(const WgradArgs& a, int mt, int nchunks, int cout_param, float* dw, hipStream_t st,
                      const BiasJob* bias = nullptr);
hipError_t prep_weights(const float* w, int cin, int cout_param, int cout, uint16_t* wt, int mpad, int kpad,
                        uint16_t* wd, int mpad_d, int kpad_d, hipStream_t st);
hipError_t prep_weights_all(const PrepJobs& jobs, hipStream_t st);
// The gradient g masked by the ReLU of act, as a packed BF16 copy (g itself
// is only read), and the bias gradient db (channels < cout_param).  part:
// FP32 scratch of BIAS_PARTS * 64 values.  defer non-null: the bias
// reduction is not launched but described in *defer (for conv_wgrad); part
// must then stay untouched until it runs.
hipError_t grad_relu_cast(const float* g, int ldg, int offg, const uint16_t* act, int lda, int offa, int c,
                          int64_t total, uint16_t* out, float* part, int cout_param, float* db, hipStream_t st,
                          BiasJob* defer = nullptr);
hipError_t cast_input(const float* x, int64_t count, uint16_t* out, hipStream_t st);
hipError_t avgpool_fwd(const uint16_t* x, int ld, int off, int c, int n, int d, int h, int w, uint16_t* y,
                       hipStream_t st);
hipError_t avgpool_bwd_add(const float* gy, int c, int n, int d, int h, int w, float* g, int ld, int off,
                           hipStream_t st);
hipError_t upsample_fwd(const uint16_t* x, int c, int n, int d, int h, int w, uint16_t* y, hipStream_t st);
hipError_t upsample_bwd(const float* gy, int c, int n, int d, int h, int w, float* g, hipStream_t st);
hipError_t trilinear(const float* x, int n, int d, int h, int w, float* y, int ldo, hipStream_t st);
hipError_t add_residual(const float* base, const float* r, int64_t total, float* out, hipStream_t st);
hipError_t loss_and_grad(const float* base, const float* r, const float* target, const uint8_t* mask, int64_t total,
                         double* part, double* stats, float* dr, hipStream_t st);
hipError_t adam(float* w, const float* g, float* m, float* v, int64_t count, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t st);
hipError_t crop(const float* uc, const uint8_t* mc, int Dc, int Hc, int Wc, const float* uf, const uint8_t* mf,
                const int* origin, int n, int d, int h, int w, int margin, float* xin, float* tgt, uint8_t* tmask,
                hipStream_t st);
hipError_t scatter(const double* vals, const int32_t* xyz, int64_t count, int D, int H, int W, double scale,
                   float* dense, uint8_t* mask, hipStream_t st);
hipError_t gather(const float* dense, const int32_t* xyz, int64_t count, int D, int H, int W, double scale,
                  double* vals, hipStream_t st);
hipError_t fill(void* p, size_t bytes, uint32_t value, hipStream_t st);

}  // namespace lbmnet_dev
