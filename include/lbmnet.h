/*
 * lbmnet.h -- C ABI of the learned coarse-to-fine velocity corrector.
 *
 * Context: Sec. 3.4 compares a simulation at twice the grid spacing (and,
 * with acoustic scaling, twice the time step) with the fine one and scores the
 * agreement of their velocity fields with a similarity index (Eq. (11)).  This
 * module maps the period-averaged velocity of such a coarse run to the fine
 * grid with a small 3D convolutional U-net that predicts a residual over the
 * trilinear upsampling of the coarse field.  It is an addition to the paper's
 * method, trained and run on the GPU with the kernels of this library.
 *
 * Network (coarse grid d x h x w, fine grid 2d x 2h x 2w; every convolution
 * is 3x3x3, stride 1, zero padded; ReLU after every layer but the head):
 *   x = (u_c (3 components), fluid mask_c)                      coarse, 4 ch
 *   e1 = conv e1b(conv e1a(x))                       4 -> 16 -> 16, coarse
 *   e2 = conv e2c(conv e2b(conv e2a(avgpool2(e1))))  16 -> 32 -> 32 -> 32, half
 *   u1 = conv u1(upsample2(e2))                      32 -> 16, coarse
 *   d1 = conv d1b(conv d1a(concat(e1, u1)))          32 -> 16 -> 16, coarse
 *   r  = head(conv f2(conv f1(upsample2(d1))))       16 -> 16 -> 16 -> 3, fine
 *   out = trilinear2(u_c) + r                                   fine, 3 ch
 * avgpool2 is 2x2x2 averaging, upsample2 nearest-neighbour 2x, and trilinear2
 * puts fine node 2i on coarse node i, odd fine nodes at the mean of their
 * coarse neighbours and repeats the last coarse node past the upper face.
 *
 * Parameters: one FP32 array, layers in the order above (e1a, e1b, e2a, e2b,
 * e2c, u1, d1a, d1b, f1, f2, head), each as weights [c_out][27][c_in] (tap =
 * 9 (dz + 1) + 3 (dy + 1) + (dx + 1), cross-correlation) followed by the bias
 * [c_out]; 127,651 values.
 *
 * Precision: FP32 master weights, Adam moments and gradients; convolutions
 * on the matrix cores with BF16 operands (weights and activations rounded to
 * nearest even) and FP32 accumulation; activations stored in BF16 between
 * layers; the head output, the trilinear base, the loss and every gradient
 * buffer are FP32; the loss sum is FP64.  All reductions run in a fixed
 * order, so results are bitwise deterministic.
 *
 * Tensors are channels-last: element (sample s, voxel (z, y, x), channel c)
 * of a tensor with C channels sits at [((s * D + z) * H + y) * W + x][c].
 *
 * Conventions (as in lbm.h): return LBM_OK or a negative LBM_E* code with a
 * message in lbm_last_error(); the library never allocates GPU memory (the
 * caller attaches a buffer of lbmnet_device_bytes); work is asynchronous on
 * the stream given at creation unless stated; a network object is not
 * thread-safe.
 */
#ifndef LBMNET_H
#define LBMNET_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbmnet lbmnet;   /* opaque, library-owned */

enum { LBMNET_LAYERS = 11 };

/* Number of parameters (127,651). */
int lbmnet_param_count(int64_t* n);

/* Layer i (0..10): info = { c_in, c_out, relu (0/1), level (0 coarse,
 * 1 half, 2 fine), offset of its weights in the parameter array }. */
int lbmnet_layer_info(int i, int64_t info[5]);

/* A network for batches of n samples of coarse size d x h x w (fine 2d x 2h
 * x 2w).  d and h must be even and w a multiple of 32; train = 1 also plans
 * the gradient, optimizer and loss buffers.  EINVAL for bad sizes. */
int lbmnet_create(int n, int d, int h, int w, int train, void* hip_stream, lbmnet** out);

/* Device bytes lbmnet_attach_device needs. */
int lbmnet_device_bytes(const lbmnet* net, size_t* bytes);

/* Attach caller-owned device memory (256-byte aligned, at least
 * lbmnet_device_bytes).  ENOMEM if too small, EINVAL if misaligned. */
int lbmnet_attach_device(lbmnet* net, void* dev_ptr, size_t bytes);

/* Upload the parameters (host FP32, lbmnet_param_count values), reset the
 * Adam moments and step counter.  Synchronizes the stream.  EINVAL if a
 * value is not finite. */
int lbmnet_set_params(lbmnet* net, const float* params);

/* Download the FP32 master parameters (host).  Synchronizes the stream. */
int lbmnet_get_params(lbmnet* net, float* params);

/* Inference: x device FP32 [n][d][h][w][4] -> out device FP32
 * [n][2d][2h][2w][3].  ESTATE before parameters are set. */
int lbmnet_forward(lbmnet* net, const float* x, float* out);

/* Forward, masked mean squared error against target (device FP32
 * [n][2d][2h][2w][3]) over the voxels where mask (device uint8, same grid)
 * is non-zero (mean over those voxels and the 3 components), and the
 * gradient of that loss with respect to every parameter (kept inside for
 * lbmnet_adam_step, also copied to grad when grad is a device FP32 array of
 * lbmnet_param_count values, else NULL).  loss: host double, written after a
 * stream synchronization when non-NULL (NULL keeps the call asynchronous).
 * ESTATE unless created with train = 1 and parameters are set. */
int lbmnet_loss_grad(lbmnet* net, const float* x, const float* target, const uint8_t* mask, double* loss,
                     float* grad);

/* One Adam step (Kingma and Ba, bias-corrected moments) on the FP32 master
 * parameters with the gradient of the last lbmnet_loss_grad.  EINVAL unless
 * lr > 0, 0 <= b1, b2 < 1, eps >= 0; ESTATE without a gradient. */
int lbmnet_adam_step(lbmnet* net, float lr, float b1, float b2, float eps);

/* Number of Adam steps taken since the parameters were set. */
int lbmnet_adam_count(const lbmnet* net, int64_t* t);

int lbmnet_destroy(lbmnet* net);

/* ---- one convolution layer, for checking the kernels on their own ----------
 * y = conv(bf16(x), bf16(w)) + b, then ReLU when relu = 1, as FP32 (the
 * network stores it in BF16).  With dy non-NULL also the backward of that
 * layer: dz = dy * [bf16(y) > 0] (or dy without ReLU), db = sum over voxels of dz
 * (FP32), dw = correlation of bf16(dz) with bf16(x), dx = the transposed
 * convolution of bf16(dz) with bf16(w); FP32 accumulation throughout.
 * x [n][d][h][w][cin], w [cout][27][cin], b [cout], dy and y [..][cout],
 * dx like x, dw like w, db like b: device FP32.  cin a multiple of 4 and at
 * most 32, cout one of 4, 8, 16, 32, w a multiple of 16.  work: device scratch of
 * lbmnet_conv3d_workspace bytes, 256-byte aligned.  Asynchronous. */
int lbmnet_conv3d_workspace(int n, int d, int h, int w, int cin, int cout, size_t* bytes);
int lbmnet_conv3d(int n, int d, int h, int w, int cin, int cout, int relu, const float* x, const float* wts,
                  const float* b, const float* dy, float* y, float* dx, float* dw, float* db, void* work,
                  size_t work_bytes, void* hip_stream);

/* ---- the same layer for callers that cannot allocate ----------------------
 * For code under HIP graph capture, tight serving loops and harnesses that
 * forbid device allocation: lbmnet_conv3d with the same arguments and results
 * (the same kernels, bit for bit), but its workspace is a fixed 64 MiB device
 * array of the library (lbmnet_conv3d_noalloc_limit reports the size) that
 * each GPU holds from the first call on it until the process ends.  The call
 * allocates nothing.  EINVAL (nothing launched) when the layer's
 * lbmnet_conv3d_workspace exceeds the limit; EDEVICE if the array's device
 * address cannot be found.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (different streams or host threads without
 * ordering) race and give wrong results; calls ordered on one stream are safe.
 * The array keeps the last call's contents; nothing in it needs clearing
 * between calls. */
int lbmnet_conv3d_noalloc_limit(size_t* bytes);
int lbmnet_conv3d_noalloc(int n, int d, int h, int w, int cin, int cout, int relu, const float* x,
                          const float* wts, const float* b, const float* dy, float* y, float* dx, float* dw,
                          float* db, void* hip_stream);

/* ---- data movement between node lists and dense grids ----------------------
 * Scatter: dense (device FP32 [D][H][W][3]) and mask (device uint8 [D][H][W])
 * are cleared, then for node i with coordinates xyz[i] = (x, y, z) (device
 * int32 [count][3]) dense[z][y][x][c] = scale * vals[c][i] (vals device FP64
 * [3][count]; product in FP64, rounded to FP32) and mask = 1.  Nodes outside
 * the grid are skipped.  EINVAL for a non-finite scale. */
int lbmnet_scatter(const double* vals, const int32_t* xyz, int64_t count, int D, int H, int W, double scale,
                   float* dense, uint8_t* mask, void* hip_stream);

/* Gather: vals[c][i] = scale * dense[z][y][x][c] in FP64 (0 outside the grid). */
int lbmnet_gather(const float* dense, const int32_t* xyz, int64_t count, int D, int H, int W, double scale,
                  double* vals, void* hip_stream);

/* Crops for training and inference.  For sample s with coarse origin o =
 * origins[s] (device int32 [n][3] as (z, y, x)): xin[s][z][y][x] = (u_c,
 * mask_c) at coarse o + (z, y, x) (zeros outside the coarse grid Dc x Hc x
 * Wc), target[s][Z][Y][X] = u_f at fine 2 o + (Z, Y, X) (fine grid 2Dc x 2Hc
 * x 2Wc) and tmask = fine mask there, cleared within `margin` voxels of a crop
 * face.  uc: FP32 [Dc][Hc][Wc][3], mc uint8 [Dc][Hc][Wc]; uf, mf on the fine
 * grid.  xin [n][d][h][w][4], target [n][2d][2h][2w][3], tmask uint8. */
int lbmnet_crop(const float* uc, const uint8_t* mc, int Dc, int Hc, int Wc, const float* uf, const uint8_t* mf,
                const int32_t* origins, int n, int d, int h, int w, int margin, float* xin, float* target,
                uint8_t* tmask, void* hip_stream);

/* The trilinear base alone: out (device FP32 [n][2d][2h][2w][3]) =
 * trilinear2 of the first 3 channels of x (device FP32 [n][d][h][w][4]). */
int lbmnet_trilinear(const float* x, int n, int d, int h, int w, float* out, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBMNET_H */
