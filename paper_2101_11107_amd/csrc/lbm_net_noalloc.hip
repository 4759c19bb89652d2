// lbmnet_conv3d_noalloc: the single-layer convolution entry point of
// lbmnet.h with its workspace taken from a fixed device array of this library
// instead of a caller buffer, for callers that cannot allocate device memory.
//
// The workspace (BF16 copies of the input, the output and its gradient, the
// packed weights, weight- and bias-gradient partials) lives in `scratch`, a
// file-scope device array that every GPU the library runs on holds until the
// process ends.  In host code `scratch` names a host-side stand-in, not the
// device array: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to the kernels.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "lbm_host.h"
#include "lbmnet.h"

namespace {

constexpr size_t SCRATCH_BYTES = size_t(64) << 20;   // 64 MiB per device
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first
// call there).  Returns a negative LBM code on failure.
int scratch_address(void** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev), "lbmnet_conv3d_noalloc: current device");
    if (dev < 0 || dev >= MAX_DEVICES) return lbm_host::fail(LBM_EDEVICE, "lbmnet_conv3d_noalloc: device index");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "lbmnet_conv3d_noalloc: scratch address");
        if (p == nullptr) return lbm_host::fail(LBM_EDEVICE, "lbmnet_conv3d_noalloc: no scratch address");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return LBM_OK;
}

}  // namespace

extern "C" int lbmnet_conv3d_noalloc_limit(size_t* bytes) {
    if (!bytes) return LBM_EINVAL;
    *bytes = SCRATCH_BYTES;
    return LBM_OK;
}

extern "C" int lbmnet_conv3d_noalloc(int n, int d, int h, int w, int cin, int cout, int relu, const float* x,
                                     const float* wts, const float* b, const float* dy, float* y, float* dx,
                                     float* dw, float* db, void* hip_stream) {
    size_t need = 0;
    int rc = lbmnet_conv3d_workspace(n, d, h, w, cin, cout, &need);   // sets the message on EINVAL
    if (rc) return rc;
    if (need > SCRATCH_BYTES)
        return lbm_host::fail(LBM_EINVAL, "lbmnet_conv3d_noalloc: the layer needs " + std::to_string(need) +
                                              " bytes of workspace, more than the fixed " +
                                              std::to_string(SCRATCH_BYTES) + " (use lbmnet_conv3d)");
    void* base = nullptr;
    rc = scratch_address(&base);
    if (rc) return rc;
    // The workspace needs no clearing: every kernel writes the parts of it
    // that a later kernel of the same call reads.
    return lbmnet_conv3d(n, d, h, w, cin, cout, relu, x, wts, b, dy, y, dx, dw, db, base, SCRATCH_BYTES,
                         hip_stream);
}
