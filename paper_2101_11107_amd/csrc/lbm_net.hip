// HIP kernels of the learned coarse-to-fine velocity corrector (gfx950).
//
// Tensors are channels-last: element (sample s, voxel v, channel c) of a
// tensor with row length ld sits at [(s * V + v) * ld + c], V = D * H * W and
// v = (z * H + y) * W + x.  Convolutions are 3x3x3, stride 1, zero padded,
// computed as implicit GEMMs on the matrix cores with
// v_mfma_f32_16x16x16bf16_1k: BF16 operands, FP32 accumulation.  Lane l of a
// wavefront holds A[l % 16][4 (l / 16) + j], B[4 (l / 16) + j][l % 16] and
// D[4 (l / 16) + j][l % 16], j = 0..3.
//
// Forward:  Y[v][co] = b[co] + sum_{tap, ci} W[co][tap][ci] X[v + off(tap)][ci]
//           (M = output channels, N = voxels, K = 27 * input channels ordered
//           tap-major, so four consecutive K are four consecutive channels of
//           one voxel: one 8-byte load per lane).
// Gradient with respect to the input: the same kernel with the weights
//           flipped in the taps and transposed in the channels.
// Gradient with respect to the weights: M = output channels, N = (tap,
//           input channel), K = voxels; per-chunk partial sums reduced in a
//           fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lbm_net_internal.h"

namespace lbmnet_dev {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8b __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    const __bf16 h = (__bf16)f;                // round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float bf2f(uint16_t h) {
    return __builtin_bit_cast(float, (uint32_t)h << 16);
}

constexpr int CONV_WAVES = 4;   // waves per work-group
constexpr int CONV_VOX = 32;    // voxels per wave (two 16-voxel tiles in one row)

// --- convolution forward (also used for the input gradient) --------------------
template <int MT, bool F32OUT>
__global__ __launch_bounds__(CONV_WAVES * 64) void k_conv_fwd(ConvArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, r16 = lane & 15;
    const int64_t V = (int64_t)a.d * a.h * a.w;
    const int64_t total = (int64_t)a.n * V;
    const int64_t vbase = ((int64_t)blockIdx.x * CONV_WAVES + wave) * CONV_VOX;
    if (vbase >= total) return;
    // each 16-voxel tile lies in one row (w is a multiple of 16): row coordinates are wave-uniform
    int s[2], z[2], y[2], x[2];
    bool valid[2];
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        const int64_t v0 = vbase + nt * 16;
        valid[nt] = v0 < total;
        const int64_t vv = valid[nt] ? v0 : 0;
        s[nt] = (int)(vv / V);
        const int64_t rr = vv - (int64_t)s[nt] * V;
        z[nt] = (int)(rr / ((int64_t)a.h * a.w));
        y[nt] = (int)((rr / a.w) % a.h);
        x[nt] = (int)(rr % a.w) + r16;
    }
    v4f acc[MT][2];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) acc[mt][nt] = v4f{0.f, 0.f, 0.f, 0.f};
    const int K = 27 * a.cin;
    for (int k0 = 0; k0 < a.kpad; k0 += 16) {
        const int k = k0 + 4 * q;
        const int tap = k / a.cin, ci = k - tap * a.cin;
        const bool kin = k < K;
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        v4s b[2];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int zz = z[nt] + dz, yy = y[nt] + dy, xx = x[nt] + dx;
            const bool ok = kin && valid[nt] && zz >= 0 && zz < a.d && yy >= 0 && yy < a.h && xx >= 0 && xx < a.w;
            const int64_t vox = ((int64_t)s[nt] * V + ((int64_t)zz * a.h + yy) * a.w + xx);
            b[nt] = ok ? *(const v4s*)(a.x + vox * a.ldx + a.cxo + ci) : v4s{0, 0, 0, 0};
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const v4s aw = *(const v4s*)(a.wt + (int64_t)(mt * 16 + r16) * a.kpad + k);
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
                acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aw, b[nt], acc[mt][nt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
        if (!valid[nt]) continue;
        const int64_t vox = vbase + nt * 16 + r16;
        if (vox >= total) continue;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int co = mt * 16 + 4 * q + j;
                if (co >= a.cout) continue;
                float val = acc[mt][nt][j] + (a.bias ? a.bias[co] : 0.0f);
                if (a.relu) val = val > 0.0f ? val : 0.0f;
                const int64_t idx = vox * a.ldy + a.cyo + co;
                if (F32OUT) ((float*)a.y)[idx] = val;
                else ((uint16_t*)a.y)[idx] = f2bf(val);
            }
        }
    }
}

// --- convolution forward on a brick staged in LDS -----------------------------------
// A work-group computes a 16 x 4 x 4 (x, y, z) brick of output voxels (16
// N-tiles of 16 voxels, four per wave).  The 18 x 6 x 6 input halo is first
// copied to LDS with 8- or 16-byte loads (zeros outside the grid), so the B
// fragments come from LDS; the weights (A) stay in global memory, where the
// L1 serves them to every wave.  Requires d % 4 == 0, h % 4 == 0, w % 16 == 0.
constexpr int BX = 16, BY = 4, BZ = 4;
constexpr int HX = BX + 2, HY = BY + 2, HZ = BZ + 2;

template <int CIN, int MT, bool F32OUT>
__global__ __launch_bounds__(256) void k_conv_fwd_lds(ConvArgs a) {
    constexpr int PIECE = CIN * 2 >= 16 ? 16 : CIN * 2;   // bytes per staging load
    constexpr int PPV = CIN * 2 / PIECE;                   // pieces per voxel
    constexpr int NHALO = HZ * HY * HX;
    __shared__ __attribute__((aligned(16))) uint16_t tile[NHALO * CIN];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, r16 = lane & 15;
    const int tx = a.w / BX, ty = a.h / BY, tz = a.d / BZ;
    int b = blockIdx.x;
    const int bx = b % tx;
    b /= tx;
    const int by = b % ty;
    b /= ty;
    const int bz = b % tz;
    const int s = b / tz;
    const int xs = bx * BX - 1, ys = by * BY - 1, zs = bz * BZ - 1;   // halo origin
    const int64_t V = (int64_t)a.d * a.h * a.w;
    const int64_t sbase = (int64_t)s * V;
    // every staging load of the thread is issued before the first LDS store
    constexpr int HITER = (NHALO * PPV + 255) / 256;
    using Piece = typename std::conditional<PIECE == 16, uint4, uint2>::type;
    Piece pc[HITER];
#pragma unroll
    for (int i = 0; i < HITER; ++i) {
        const int idx = (int)threadIdx.x + 256 * i;
        const int vox = idx / PPV, p = idx - vox * PPV;
        const int hx = vox % HX, hy = (vox / HX) % HY, hz = vox / (HX * HY);
        const int xx = xs + hx, yy = ys + hy, zz = zs + hz;
        const bool in = idx < NHALO * PPV && xx >= 0 && xx < a.w && yy >= 0 && yy < a.h && zz >= 0 && zz < a.d;
        const uint16_t* src = a.x + (sbase + ((int64_t)zz * a.h + yy) * a.w + xx) * a.ldx + a.cxo + p * (PIECE / 2);
        pc[i] = in ? *(const Piece*)src : Piece{};
    }
#pragma unroll
    for (int i = 0; i < HITER; ++i) {
        const int idx = (int)threadIdx.x + 256 * i;
        if (idx >= NHALO * PPV) continue;
        const int vox = idx / PPV, p = idx - vox * PPV;
        *(Piece*)(tile + vox * CIN + p * (PIECE / 2)) = pc[i];
    }
    __syncthreads();
    v4f acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[mt][t] = v4f{0.f, 0.f, 0.f, 0.f};
    constexpr int K = 27 * CIN;
    // wave: output plane z = wave; N-tile t: output row y = t, x = r16
    if constexpr (CIN % 8 == 0) {
        // v_mfma_f32_16x16x32_bf16: a lane holds 8 consecutive K, i.e. 8
        // channels of one tap (one 16-byte read each for A and B)
        constexpr int KP32 = (K + 31) / 32 * 32;
#pragma unroll (CIN >= 32 ? 3 : 14)
        for (int k0 = 0; k0 < KP32; k0 += 32) {
            const int k = k0 + 8 * q;
            const int tap = k / CIN, ci = k - tap * CIN;
            const bool kin = k < K;
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;   // offsets + 1
            v8b aw[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                const v8b z = {};
                aw[mt] = kin ? *(const v8b*)(a.wt + (int64_t)(mt * 16 + r16) * a.kpad + k) : z;
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int hv = ((wave + dz) * HY + (t + dy)) * HX + (r16 + dx);
                const v8b z = {};
                const v8b bv = kin ? *(const v8b*)(tile + hv * CIN + ci) : z;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aw[mt], bv, acc[mt][t], 0, 0, 0);
            }
        }
    } else {
        constexpr int KPAD = (K + 15) / 16 * 16;
#pragma unroll
        for (int k0 = 0; k0 < KPAD; k0 += 16) {
            const int k = k0 + 4 * q;
            const int tap = k / CIN, ci = k - tap * CIN;
            const bool kin = k < K;
            const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;   // offsets + 1
            v4s aw[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) aw[mt] = *(const v4s*)(a.wt + (int64_t)(mt * 16 + r16) * a.kpad + k);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int hv = ((wave + dz) * HY + (t + dy)) * HX + (r16 + dx);
                const v4s bv = kin ? *(const v4s*)(tile + hv * CIN + ci) : v4s{0, 0, 0, 0};
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(aw[mt], bv, acc[mt][t], 0, 0, 0);
            }
        }
    }
    // a lane holds channels 4q .. 4q + 3 of one voxel: one 16-byte (FP32) or
    // 8-byte (BF16) store when they are aligned and all valid or all absent
    const bool vec = a.cout % 4 == 0 && a.ldy % 4 == 0 && a.cyo % 4 == 0 &&
                     ((uintptr_t)a.y & (F32OUT ? 15 : 7)) == 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t vox = sbase + ((int64_t)(zs + 1 + wave) * a.h + (ys + 1 + t)) * a.w + (xs + 1 + r16);
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int co0 = mt * 16 + 4 * q;
            float val[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int co = co0 + j;
                val[j] = acc[mt][t][j] + (a.bias && co < a.cout ? a.bias[co] : 0.0f);
                if (a.relu) val[j] = val[j] > 0.0f ? val[j] : 0.0f;
            }
            const int64_t idx0 = vox * a.ldy + a.cyo + co0;
            if (vec) {
                if (co0 >= a.cout) continue;
                if (F32OUT) {
                    *(float4*)((float*)a.y + idx0) = float4{val[0], val[1], val[2], val[3]};
                } else {
                    const uint32_t lo = (uint32_t)f2bf(val[0]) | ((uint32_t)f2bf(val[1]) << 16);
                    const uint32_t hi = (uint32_t)f2bf(val[2]) | ((uint32_t)f2bf(val[3]) << 16);
                    *(uint2*)((uint16_t*)a.y + idx0) = uint2{lo, hi};
                }
                continue;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (co0 + j >= a.cout) continue;
                if (F32OUT) ((float*)a.y)[idx0 + j] = val[j];
                else ((uint16_t*)a.y)[idx0 + j] = f2bf(val[j]);
            }
        }
    }
}

// --- weight gradient ------------------------------------------------------------
// Block: one chunk of voxels (blockIdx.x) and 16 N-tiles (blockIdx.y), 4 per wave.
template <int MT>
__global__ __launch_bounds__(256) void k_conv_wgrad(WgradArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, r16 = lane & 15;
    const int64_t V = (int64_t)a.d * a.h * a.w;
    const int64_t total = (int64_t)a.n * V;
    const int N = 27 * a.cin;
    const int ntile0 = blockIdx.y * 16 + wave * 4;
    int tapn[4], cin_n[4];
    bool nin[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int n = (ntile0 + t) * 16 + r16;
        nin[t] = n < N;
        tapn[t] = nin[t] ? n / a.cin : 0;
        cin_n[t] = nin[t] ? n - tapn[t] * a.cin : 0;
    }
    v4f acc[MT][4];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[mt][t] = v4f{0.f, 0.f, 0.f, 0.f};
    const int64_t c0 = (int64_t)blockIdx.x * a.chunk;
    const int64_t c1 = c0 + a.chunk < total ? c0 + a.chunk : total;
    for (int64_t k0 = c0; k0 < c1; k0 += 16) {
        // 16 voxels in one row: wave-uniform row coordinates
        const int s = (int)(k0 / V);
        const int64_t rr = k0 - (int64_t)s * V;
        const int z = (int)(rr / ((int64_t)a.h * a.w));
        const int y = (int)((rr / a.w) % a.h);
        const int x0 = (int)(rr % a.w) + 4 * q;
        v4s am[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int co = mt * 16 + r16;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                am[mt][j] = (co < a.cout) ? (short)a.dy[(k0 + 4 * q + j) * a.ldy + co] : (short)0;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int tap = tapn[t];
            const int dz = tap / 9 - 1, dyy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
            const int zz = z + dz, yy = y + dyy;
            const bool rowok = nin[t] && zz >= 0 && zz < a.d && yy >= 0 && yy < a.h;
            const int64_t rowbase = ((int64_t)s * V + ((int64_t)zz * a.h + yy) * a.w);
            v4s bn;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int xx = x0 + j + dx;
                const bool ok = rowok && xx >= 0 && xx < a.w;
                bn[j] = ok ? (short)a.x[(rowbase + xx) * a.ldx + a.cxo + cin_n[t]] : (short)0;
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am[mt], bn, acc[mt][t], 0, 0, 0);
        }
    }
    float* part = a.part + (int64_t)blockIdx.x * a.mpad * a.npad;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int n = (ntile0 + t) * 16 + r16;
            if (n >= a.npad) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) part[(mt * 16 + 4 * q + j) * a.npad + n] = acc[mt][t][j];
        }
}

// --- weight gradient on bricks staged in LDS ---------------------------------------
// Work-group (p, yb) accumulates, over the bricks p, p + P, p + 2P, ..., the
// contribution of every voxel of the brick to N-tiles 28 yb .. 28 yb + 27 (7
// per wave) and writes one partial per work-group.  Per brick the input halo
// goes to LDS channel-major ([ci][halo voxel]) and the output gradient
// transposed ([co][brick voxel]), so an A fragment (4 voxels of one channel)
// is one 8-byte read and a B fragment 4 consecutive 2-byte reads.  The global
// loads of the next brick are issued into registers before the MFMA loop of
// the current one, so their latency hides behind it (a work-group handles
// many bricks in turn and only a few work-groups share a CU).
constexpr int WG_TPW = 7;   // N-tiles per wave

template <int PIECE>
struct HaloPiece {
    uint2 v;
};
template <>
struct HaloPiece<16> {
    uint4 v;
};

template <int CIN, int MT>
__global__ __launch_bounds__(256) void k_conv_wgrad_lds(WgradArgs a, int nparts) {
    constexpr int PIECE = CIN * 2 >= 16 ? 16 : CIN * 2;
    constexpr int PPV = CIN * 2 / PIECE;
    constexpr int NHALO = HZ * HY * HX;
    constexpr int NB = BX * BY * BZ;   // voxels per brick (256, one per thread)
    constexpr int N = 27 * CIN;
    constexpr int HITER = (NHALO * PPV + 255) / 256;   // halo pieces per thread
    constexpr int GQ = 4 * MT;                           // 4-channel gradient pieces per voxel, at most
    __shared__ __attribute__((aligned(16))) uint16_t halo[CIN * NHALO];
    __shared__ __attribute__((aligned(16))) uint16_t gy[MT * 16 * NB];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, r16 = lane & 15;
    const int tx = a.w / BX, ty = a.h / BY, tz = a.d / BZ;
    const int64_t nbricks = (int64_t)a.n * tx * ty * tz;
    const int64_t V = (int64_t)a.d * a.h * a.w;
    const int gq = a.cout >> 2;
    // rows of the output gradient beyond cout stay zero
    for (int k = threadIdx.x; k < MT * 16 * NB; k += 256) gy[k] = 0;
    // this wave's N-tiles: column n -> (tap, ci)
    int tap_of[WG_TPW], ci_of[WG_TPW];
    bool nin[WG_TPW];
#pragma unroll
    for (int t = 0; t < WG_TPW; ++t) {
        const int n = ((int)blockIdx.y * 4 * WG_TPW + wave * WG_TPW + t) * 16 + r16;
        nin[t] = n < N;
        tap_of[t] = nin[t] ? n / CIN : 0;
        ci_of[t] = nin[t] ? n - tap_of[t] * CIN : 0;
    }
    v4f acc[MT][WG_TPW];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int t = 0; t < WG_TPW; ++t) acc[mt][t] = v4f{0.f, 0.f, 0.f, 0.f};

    // Global loads of brick br into registers: halo pieces idx = tid + 256 i
    // (voxel idx / PPV, piece idx % PPV; zeros outside the grid) and the
    // gradient of brick voxel tid (cout / 4 pieces of 4 channels).
    HaloPiece<PIECE> hreg[HITER];
    uint2 greg[GQ];
    auto fetch = [&](int64_t br) {
        int64_t b = br;
        const int bx = (int)(b % tx);
        b /= tx;
        const int by = (int)(b % ty);
        b /= ty;
        const int bz = (int)(b % tz);
        const int s = (int)(b / tz);
        const int xs = bx * BX - 1, ys = by * BY - 1, zs = bz * BZ - 1;
        const int64_t sbase = (int64_t)s * V;
#pragma unroll
        for (int i = 0; i < HITER; ++i) {
            const int idx = (int)threadIdx.x + 256 * i;
            const int vox = idx / PPV, p = idx - vox * PPV;
            const int hx = vox % HX, hy = (vox / HX) % HY, hz = vox / (HX * HY);
            const int xx = xs + hx, yy = ys + hy, zz = zs + hz;
            const bool in = idx < NHALO * PPV && xx >= 0 && xx < a.w && yy >= 0 && yy < a.h && zz >= 0 && zz < a.d;
            const uint16_t* src =
                a.x + (sbase + ((int64_t)zz * a.h + yy) * a.w + xx) * a.ldx + a.cxo + p * (PIECE / 2);
            if constexpr (PIECE == 16) hreg[i].v = in ? *(const uint4*)src : uint4{0u, 0u, 0u, 0u};
            else hreg[i].v = in ? *(const uint2*)src : uint2{0u, 0u};
        }
        const int v = threadIdx.x;
        const int vx = v % BX, vy = (v / BX) % BY, vz = v / (BX * BY);
        const int64_t g = sbase + ((int64_t)(zs + 1 + vz) * a.h + (ys + 1 + vy)) * a.w + (xs + 1 + vx);
        const uint2* gsrc = (const uint2*)(a.dy + g * a.ldy);
#pragma unroll
        for (int k = 0; k < GQ; ++k) greg[k] = k < gq ? gsrc[k] : uint2{0u, 0u};
    };
    // Registers -> LDS, with the layouts the fragments read.
    auto stage = [&]() {
#pragma unroll
        for (int i = 0; i < HITER; ++i) {
            const int idx = (int)threadIdx.x + 256 * i;
            if (idx >= NHALO * PPV) continue;
            const int vox = idx / PPV, p = idx - vox * PPV;
            uint32_t ww[PIECE / 4];
            if constexpr (PIECE == 16) {
                ww[0] = hreg[i].v.x, ww[1] = hreg[i].v.y, ww[2] = hreg[i].v.z, ww[3] = hreg[i].v.w;
            } else {
                ww[0] = hreg[i].v.x, ww[1] = hreg[i].v.y;
            }
#pragma unroll
            for (int e = 0; e < PIECE / 4; ++e) {
                halo[(p * (PIECE / 2) + 2 * e) * NHALO + vox] = (uint16_t)(ww[e] & 0xffffu);
                halo[(p * (PIECE / 2) + 2 * e + 1) * NHALO + vox] = (uint16_t)(ww[e] >> 16);
            }
        }
        const int v = threadIdx.x;
#pragma unroll
        for (int k = 0; k < GQ; ++k) {
            if (k >= gq) continue;
            gy[(4 * k + 0) * NB + v] = (uint16_t)(greg[k].x & 0xffffu);
            gy[(4 * k + 1) * NB + v] = (uint16_t)(greg[k].x >> 16);
            gy[(4 * k + 2) * NB + v] = (uint16_t)(greg[k].y & 0xffffu);
            gy[(4 * k + 3) * NB + v] = (uint16_t)(greg[k].y >> 16);
        }
    };

    int64_t br = blockIdx.x;
    if (br < nbricks) fetch(br);
    for (; br < nbricks; br += nparts) {
        __syncthreads();   // the previous brick's fragments have been read
        stage();
        __syncthreads();
        if (br + nparts < nbricks) fetch(br + nparts);
#pragma unroll 2
        for (int k0 = 0; k0 < NB; k0 += 16) {
            const int v0 = k0 + 4 * q;   // 4 voxels of one x row of the brick
            const int vx = v0 % BX, vy = (v0 / BX) % BY, vz = v0 / (BX * BY);
            v4s am[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) am[mt] = *(const v4s*)(gy + (mt * 16 + r16) * NB + v0);
#pragma unroll
            for (int t = 0; t < WG_TPW; ++t) {
                const int tap = tap_of[t];
                const int hv = ((vz + tap / 9) * HY + (vy + (tap / 3) % 3)) * HX + (vx + tap % 3);
                const uint16_t* hp = halo + ci_of[t] * NHALO + hv;
                v4s bn;
#pragma unroll
                for (int j = 0; j < 4; ++j) bn[j] = nin[t] ? (short)hp[j] : (short)0;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am[mt], bn, acc[mt][t], 0, 0, 0);
            }
        }
    }
    float* part = a.part + (int64_t)blockIdx.x * a.mpad * a.npad;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int t = 0; t < WG_TPW; ++t) {
            const int n = ((int)blockIdx.y * 4 * WG_TPW + wave * WG_TPW + t) * 16 + r16;
            if (n >= a.npad) continue;
#pragma unroll
            for (int j = 0; j < 4; ++j) part[(mt * 16 + 4 * q + j) * a.npad + n] = acc[mt][t][j];
        }
}

// --- weight gradient, 16 x 16 channel tiles, waves split the brick --------------
// For cin a multiple of 16 and cout <= 16 MT.  Work-group (p, y) covers input
// channels 16 (y % (cin / 16)) + 0 .. 15, output channels 16 (y / (cin / 16))
// + 0 .. 15 and all 27 taps (27 N-tiles) over the bricks p, p + P, ...; wave
// w takes the z-slice w of every brick (64 voxels, two K-steps of 32).  For
// one (dz, dy) the B fragments of dx = 0, 1, 2 are windows of consecutive
// halo values starting at an even index, so five aligned 4-byte LDS reads
// give all three (dx = 1 by 16-bit funnel shifts).  The four waves' sums are
// added in LDS in a fixed order (wave 3, 2, 1, 0) before the partial is
// written.
//
// LDS banks (32 of 4 bytes): the halo rows of the 16 channels sit HSTR
// halves apart (HSTR / 2 = 2 mod 32 dwords) and the gradient rows GSTR
// halves apart (GSTR / 2 = 4 mod 32), and lane quarter q takes row
// y = 2 m + (q & 1), x = 8 (q >> 1): the 4-byte halo reads of 32
// consecutive lanes (channel r16, two quarters) then touch 32 different banks,
// and the 16-byte gradient reads spread evenly over the banks.  Both
// transposes write whole dwords (two voxels of one channel): the halo from
// pairs of voxels a thread loads, the gradient after a swap with the
// neighbouring lane.
template <int CIN>
__global__ __launch_bounds__(256) void k_conv_wgrad_k16(WgradArgs a, int nparts) {
    constexpr int NHALO = HZ * HY * HX;
    constexpr int NB = BX * BY * BZ;                 // voxels per brick (256, one per thread)
    constexpr int HSTR = 708;                        // halves per halo channel row (>= NHALO)
    constexpr int GSTR = 264;                        // halves per gradient channel row (>= NB)
    constexpr int NPAIR = NHALO / 2;                 // voxel pairs of one channel row
    constexpr int HITER = (2 * NPAIR + 255) / 256;   // (pair, channel half) tasks per thread
    constexpr int LDS_HALFS = 16 * HSTR + 16 * GSTR;
    static_assert(BZ == 4 && BX == 16 && BY == 4, "one z-slice per wave, four K-steps of 16 per slice");
    static_assert(HX % 2 == 0 && HSTR >= NHALO && GSTR >= NB && (HSTR / 2) % 32 == 2 && (GSTR / 2) % 32 == 4,
                  "voxel pairs stay in one halo row; row strides as the bank layout needs");
    static_assert(27 * 4 * 64 * 4 <= LDS_HALFS * 2, "the wave reduction fits in the staging space");
    __shared__ __attribute__((aligned(16))) uint16_t lds[LDS_HALFS];
    uint16_t* halo = lds;                 // [16 channels][HSTR]
    uint16_t* gy = lds + 16 * HSTR;       // [16 output channels][GSTR]
    uint32_t* halo32 = (uint32_t*)halo;
    uint32_t* gy32 = (uint32_t*)gy;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, r16 = lane & 15;
    const int tx = a.w / BX, ty = a.h / BY, tz = a.d / BZ;
    const int64_t nbricks = (int64_t)a.n * tx * ty * tz;
    const int64_t V = (int64_t)a.d * a.h * a.w;
    constexpr int CG = CIN / 16;                       // input channel groups
    const int c0 = 16 * ((int)blockIdx.y % CG);        // first input channel of this work-group
    const int co0 = 16 * ((int)blockIdx.y / CG);       // first output channel of this work-group
    const int gq = (a.cout - co0) >> 2 < 4 ? (a.cout - co0) >> 2 : 4;   // 4-channel gradient pieces
    for (int k = threadIdx.x; k < 16 * GSTR / 2; k += 256) gy32[k] = 0u;   // rows co >= cout stay zero
    v4f acc[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};

    uint4 hreg[HITER][2];   // channels 8 p .. 8 p + 7 of voxels 2 m and 2 m + 1
    uint2 greg[4];
    auto fetch = [&](int64_t br) {
        int64_t b = br;
        const int bx = (int)(b % tx);
        b /= tx;
        const int by = (int)(b % ty);
        b /= ty;
        const int bz = (int)(b % tz);
        const int s = (int)(b / tz);
        const int xs = bx * BX - 1, ys = by * BY - 1, zs = bz * BZ - 1;
        const int64_t sbase = (int64_t)s * V;
#pragma unroll
        for (int i = 0; i < HITER; ++i) {
            const int task = (int)threadIdx.x + 256 * i;
            const int p = task >= NPAIR, m = task - p * NPAIR;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int vox = 2 * m + h;
                const int hx = vox % HX, hy = (vox / HX) % HY, hz = vox / (HX * HY);
                const int xx = xs + hx, yy = ys + hy, zz = zs + hz;
                const bool in = task < 2 * NPAIR && xx >= 0 && xx < a.w && yy >= 0 && yy < a.h && zz >= 0 &&
                                zz < a.d;
                const uint16_t* src =
                    a.x + (sbase + ((int64_t)zz * a.h + yy) * a.w + xx) * a.ldx + a.cxo + c0 + 8 * p;
                hreg[i][h] = in ? *(const uint4*)src : uint4{0u, 0u, 0u, 0u};
            }
        }
        const int v = threadIdx.x;
        const int vx = v % BX, vy = (v / BX) % BY, vz = v / (BX * BY);
        const int64_t g = sbase + ((int64_t)(zs + 1 + vz) * a.h + (ys + 1 + vy)) * a.w + (xs + 1 + vx);
        const uint2* gsrc = (const uint2*)(a.dy + g * a.ldy + co0);
#pragma unroll
        for (int k = 0; k < 4; ++k) greg[k] = k < gq ? gsrc[k] : uint2{0u, 0u};
    };
    auto stage = [&]() {
#pragma unroll
        for (int i = 0; i < HITER; ++i) {
            const int task = (int)threadIdx.x + 256 * i;
            if (task >= 2 * NPAIR) continue;
            const int p = task >= NPAIR, m = task - p * NPAIR;
            const uint32_t lo[4] = {hreg[i][0].x, hreg[i][0].y, hreg[i][0].z, hreg[i][0].w};
            const uint32_t hi[4] = {hreg[i][1].x, hreg[i][1].y, hreg[i][1].z, hreg[i][1].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                // channel 8 p + 2 e from the low halves, 8 p + 2 e + 1 from the high halves
                halo32[(8 * p + 2 * e) * (HSTR / 2) + m] = (lo[e] & 0xffffu) | (hi[e] << 16);
                halo32[(8 * p + 2 * e + 1) * (HSTR / 2) + m] = (lo[e] >> 16) | (hi[e] & 0xffff0000u);
            }
        }
        // gradient: even lanes write channels 0..7, odd lanes 8..15, each as
        // dwords (voxel v & ~1 in the low half, v | 1 in the high half)
        const int v = threadIdx.x;
        const bool odd = v & 1;
        uint32_t own[8], nb[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            own[2 * k] = greg[k].x;
            own[2 * k + 1] = greg[k].y;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) nb[k] = (uint32_t)__shfl_xor((int)own[k], 1, 64);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // word k (even lane) or 4 + k (odd lane) of the 8 words, two channels each
            const uint32_t even_w = odd ? nb[4 + k] : own[k];   // the even voxel's two channels
            const uint32_t odd_w = odd ? own[4 + k] : nb[k];    // the odd voxel's two channels
            const int c = 2 * k + (odd ? 8 : 0);
            if (c < 4 * gq) {
                gy32[c * (GSTR / 2) + (v >> 1)] = (even_w & 0xffffu) | (odd_w << 16);
                gy32[(c + 1) * (GSTR / 2) + (v >> 1)] = (even_w >> 16) | (odd_w & 0xffff0000u);
            }
        }
    };

    // v_mfma_f32_16x16x32_bf16, two K-steps of 32 voxels per slice: lane
    // (q, r16) takes input channel c0 + r16 and the 8 voxels x = 8 (q >> 1) ..
    // + 7 of row y = 2 m + (q & 1) (an even halo index, so 4-byte aligned)
    const int xq = 8 * (q >> 1), yq = q & 1;
    const uint16_t* hl = halo + r16 * HSTR + (wave * HY + yq) * HX + xq;
    const uint16_t* gl = gy + r16 * GSTR + wave * (BX * BY) + yq * BX + xq;
    int64_t br = blockIdx.x;
    if (br < nbricks) fetch(br);
    for (; br < nbricks; br += nparts) {
        __syncthreads();   // the previous brick's fragments have been read
        stage();
        __syncthreads();
        if (br + nparts < nbricks) fetch(br + nparts);
        typedef uint32_t u4 __attribute__((ext_vector_type(4)));
#pragma unroll
        for (int m = 0; m < BY / 2; ++m) {   // K-step: rows 2m, 2m + 1 of slice z = wave
            const v8b am = *(const v8b*)(gl + 2 * m * BX);
#pragma unroll
            for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    // ten halo values x0 .. x0 + 9 of the row give the windows of dx = 0, 1, 2
                    const uint32_t* rw = (const uint32_t*)(hl + (dz * HY + 2 * m + dy) * HX);
                    const uint32_t e0 = rw[0], e1 = rw[1], e2 = rw[2], e3 = rw[3], e4 = rw[4];
                    const uint32_t m0 = __builtin_amdgcn_alignbit(e1, e0, 16);
                    const uint32_t m1 = __builtin_amdgcn_alignbit(e2, e1, 16);
                    const uint32_t m2 = __builtin_amdgcn_alignbit(e3, e2, 16);
                    const uint32_t m3 = __builtin_amdgcn_alignbit(e4, e3, 16);
                    const int t0 = dz * 9 + dy * 3;
                    acc[t0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        am, __builtin_bit_cast(v8b, u4{e0, e1, e2, e3}), acc[t0], 0, 0, 0);
                    acc[t0 + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        am, __builtin_bit_cast(v8b, u4{m0, m1, m2, m3}), acc[t0 + 1], 0, 0, 0);
                    acc[t0 + 2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                        am, __builtin_bit_cast(v8b, u4{e1, e2, e3, e4}), acc[t0 + 2], 0, 0, 0);
                }
        }
    }
    // sum over the waves: red[(t * 4 + j) * 64 + lane], wave 3 first
    float* red = (float*)lds;
    for (int w = 3; w >= 0; --w) {
        __syncthreads();
        if (wave != w) continue;
#pragma unroll
        for (int t = 0; t < 27; ++t)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float* r = red + (t * 4 + j) * 64 + lane;
                acc[t][j] = w == 3 ? acc[t][j] : *r + acc[t][j];
                if (w > 0) *r = acc[t][j];
            }
    }
    if (wave != 0) return;
    float* part = a.part + (int64_t)blockIdx.x * a.mpad * a.npad;
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const int n = t * CIN + c0 + r16;   // column of (tap t, input channel c0 + r16)
#pragma unroll
        for (int j = 0; j < 4; ++j) part[(co0 + 4 * q + j) * a.npad + n] = acc[t][j];
    }
}

// dW[co][n] = sum over chunks, only co < cout_param written.  A work-group
// covers 32 outputs; each of its 8 thread groups sums every 8th chunk in
// ascending order, then the 8 group sums are added in order (deterministic).
// Work-groups from wblocks on reduce the bias gradient of the same layer
// instead (channel blockIdx.x - wblocks), saving a launch.
__device__ __forceinline__ void bias_reduce_block(const float* __restrict__ part, int nparts, float* __restrict__ db,
                                                  int co);
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float* __restrict__ part, int nchunks, int mpad, int npad,
                                                      int cout_param, int N, float* __restrict__ dw, int wblocks,
                                                      const float* __restrict__ bpart, int bnparts,
                                                      float* __restrict__ db) {
    if ((int)blockIdx.x >= wblocks) {
        bias_reduce_block(bpart, bnparts, db, (int)blockIdx.x - wblocks);
        return;
    }
    __shared__ float s[8][32];
    const int lane = threadIdx.x & 31, grp = threadIdx.x >> 5;
    const int e = blockIdx.x * 32 + lane;
    const int E = cout_param * N;
    float acc = 0.0f;
    if (e < E) {
        const int co = e / N, n = e - co * N;
        const float* p = part + (int64_t)co * npad + n;
        const int64_t stride = (int64_t)mpad * npad;
        // eight partials per round, loaded before they are added (ascending order)
        for (int c0 = grp; c0 < nchunks; c0 += 64) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = c0 + 8 * u < nchunks ? p[(c0 + 8 * u) * stride] : 0.0f;
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (c0 + 8 * u < nchunks) acc += v[u];
        }
    }
    s[grp][lane] = acc;
    __syncthreads();
    if (grp == 0 && e < E) {
        float t = s[0][lane];
        for (int k = 1; k < 8; ++k) t += s[k][lane];
        dw[e] = t;
    }
}

// Bias gradient from the per-work-group channel sums of k_grad_relu_cast: one
// work-group per channel, fixed-order tree (deterministic).
__device__ __forceinline__ void bias_reduce_block(const float* __restrict__ part, int nparts, float* __restrict__ db,
                                                  int co) {
    __shared__ float s[256];
    float acc = 0.0f;
    for (int b = threadIdx.x; b < nparts; b += 256) acc += part[b * 64 + co];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[co] = s[0];
}

__global__ __launch_bounds__(256) void k_bias_reduce(const float* __restrict__ part, int nparts,
                                                     float* __restrict__ db) {
    bias_reduce_block(part, nparts, db, blockIdx.x);
}

// Packed BF16 weights from FP32 masters w[co][tap][ci] (rows co >= cout_param zero):
// forward wt[m][tap * cin + ci], input-gradient wd[ci][tap' * cout + co] = w[co][26 - tap'][ci].
__device__ __forceinline__ void prep_one(const float* __restrict__ w, int cin, int cout_param, int cout, uint16_t* wt,
                                         int mpad, int kpad, uint16_t* wd, int mpad_d, int kpad_d, int idx) {
    if (idx < mpad * kpad) {
        const int m = idx / kpad, k = idx - m * kpad;
        float v = 0.0f;
        if (m < cout_param && k < 27 * cin) v = w[(m * 27 + k / cin) * cin + k % cin];
        wt[idx] = f2bf(v);
    }
    if (wd && idx < mpad_d * kpad_d) {
        const int m = idx / kpad_d, k = idx - m * kpad_d;   // m = ci, k = tap' * cout + co
        float v = 0.0f;
        if (m < cin && k < 27 * cout) {
            const int tp = k / cout, co = k - tp * cout;
            if (co < cout_param) v = w[(co * 27 + (26 - tp)) * cin + m];
        }
        wd[idx] = f2bf(v);
    }
}

__global__ void k_prep_weights(const float* __restrict__ w, int cin, int cout_param, int cout, uint16_t* wt, int mpad,
                               int kpad, uint16_t* wd, int mpad_d, int kpad_d) {
    prep_one(w, cin, cout_param, cout, wt, mpad, kpad, wd, mpad_d, kpad_d, blockIdx.x * blockDim.x + threadIdx.x);
}

// Every layer of a network in one launch: row blockIdx.y packs layer y.
__global__ void k_prep_weights_all(PrepJobs jobs) {
    const PrepJob& p = jobs.j[blockIdx.y];
    prep_one(p.w, p.cin, p.cout_param, p.cout, p.wt, p.mpad, p.kpad, p.wd, p.mpad_d, p.kpad_d,
             blockIdx.x * blockDim.x + threadIdx.x);
}

// g (FP32, channels [off, off + c) of rows of length ld) times the ReLU mask of
// act (BF16, same layout; null: no mask), written as a packed BF16 copy
// [v][c] (g itself is only read); per work-group channel sums of the masked
// FP32 values go to
// part[block][0..c) for the bias gradient.  c divides 256 and `per` (elements
// per work-group) is a multiple of 256, so a thread always sees one channel.
__global__ __launch_bounds__(256) void k_grad_relu_cast(const float* __restrict__ g, int ldg, int offg,
                                                        const uint16_t* __restrict__ act, int lda, int offa, int c,
                                                        int64_t total, int64_t per, uint16_t* __restrict__ out,
                                                        float* __restrict__ part) {
    __shared__ float s[256];
    const int64_t E = total * c;
    const int64_t e0 = (int64_t)blockIdx.x * per;
    const int64_t e1 = e0 + per < E ? e0 + per : E;
    float acc = 0.0f;
    // c is a power of two dividing 256 and e0 a multiple of 256: the channel
    // of every element this thread visits is threadIdx.x mod c
    const int ch = threadIdx.x & (c - 1);
    const int csh = __builtin_ctz((unsigned)c);
    // four elements per round: their loads are issued before the in-place
    // stores (which the compiler may not move loads across); the sum keeps
    // ascending element order
    constexpr int U = 4;
    for (int64_t i0 = e0 + threadIdx.x; i0 < e1; i0 += 256 * U) {
        float val[U];
        bool keep[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t idx = i0 + 256 * u;
            const int64_t v = idx >> csh;
            val[u] = idx < e1 ? g[v * ldg + offg + ch] : 0.0f;
            keep[u] = !act || (idx < e1 && bf2f(act[v * lda + offa + ch]) > 0.0f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t idx = i0 + 256 * u;
            if (idx >= e1) break;
            const float x = keep[u] ? val[u] : 0.0f;
            out[idx] = f2bf(x);
            acc += x;
        }
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int st = 128; st >= c; st >>= 1) {   // partners differ by a multiple of c: same channel
        if (threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < c) part[(int64_t)blockIdx.x * 64 + threadIdx.x] = s[threadIdx.x];
}

// The same with four consecutive channels per thread (16-byte FP32 and 8-byte
// BF16 accesses): c % 4 == 0, rows and offsets multiples of 4, `per` a
// multiple of 1024, so thread t always sees channels 4t mod c .. +3.
__global__ __launch_bounds__(256) void k_grad_relu_cast4(const float* __restrict__ g, int ldg, int offg,
                                                         const uint16_t* __restrict__ act, int lda, int offa, int c,
                                                         int64_t total, int64_t per, uint16_t* __restrict__ out,
                                                         float* __restrict__ part) {
    __shared__ float s[4][256];
    const int64_t E = total * c;
    const int64_t e0 = (int64_t)blockIdx.x * per;
    const int64_t e1 = e0 + per < E ? e0 + per : E;
    const int ch0 = (4 * threadIdx.x) & (c - 1);
    const int csh = __builtin_ctz((unsigned)c);
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    constexpr int U = 2;   // rounds of loads issued before the stores
    for (int64_t i0 = e0 + 4 * threadIdx.x; i0 < e1; i0 += 1024 * U) {
        float4 val[U];
        uint2 m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t idx = i0 + 1024 * u;
            const int64_t v = idx >> csh;
            val[u] = idx < e1 ? *(const float4*)(g + v * ldg + offg + ch0) : float4{0.f, 0.f, 0.f, 0.f};
            m[u] = act && idx < e1 ? *(const uint2*)(act + v * lda + offa + ch0) : uint2{0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t idx = i0 + 1024 * u;
            if (idx >= e1) break;
            float x[4] = {val[u].x, val[u].y, val[u].z, val[u].w};
            if (act) {
                const uint16_t mk[4] = {(uint16_t)(m[u].x & 0xffffu), (uint16_t)(m[u].x >> 16),
                                        (uint16_t)(m[u].y & 0xffffu), (uint16_t)(m[u].y >> 16)};
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (!(bf2f(mk[j]) > 0.0f)) x[j] = 0.0f;
            }
            const uint32_t lo = (uint32_t)f2bf(x[0]) | ((uint32_t)f2bf(x[1]) << 16);
            const uint32_t hi = (uint32_t)f2bf(x[2]) | ((uint32_t)f2bf(x[3]) << 16);
            *(uint2*)(out + idx) = uint2{lo, hi};
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[j] += x[j];
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int st = 128; st >= c / 4; st >>= 1) {   // partners differ by a multiple of c / 4 threads
        if (threadIdx.x < st)
#pragma unroll
            for (int j = 0; j < 4; ++j) s[j][threadIdx.x] += s[j][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < c / 4)
#pragma unroll
        for (int j = 0; j < 4; ++j) part[(int64_t)blockIdx.x * 64 + 4 * threadIdx.x + j] = s[j][threadIdx.x];
}

__global__ void k_cast_input(const float* __restrict__ x, int64_t count, uint16_t* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = f2bf(x[i]);
}

// 2x2x2 average pooling of BF16 channels [off, off + c) (row ld) into packed [V/8][c].
__global__ void k_avgpool_fwd(const uint16_t* __restrict__ x, int ld, int off, int c, int n, int d, int h, int w,
                              uint16_t* __restrict__ y) {
    const int d2 = d / 2, h2 = h / 2, w2 = w / 2;
    const int64_t total = (int64_t)n * d2 * h2 * w2 * c;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    int64_t r = idx;
    const int ch = (int)(r % c); r /= c;
    const int X = (int)(r % w2); r /= w2;
    const int Y = (int)(r % h2); r /= h2;
    const int Z = (int)(r % d2);
    const int s = (int)(r / d2);
    float acc = 0.0f;
    for (int k = 0; k < 8; ++k) {
        const int64_t v = (((int64_t)s * d + 2 * Z + (k >> 2)) * h + 2 * Y + ((k >> 1) & 1)) * w + 2 * X + (k & 1);
        acc += bf2f(x[v * ld + off + ch]);
    }
    y[idx] = f2bf(acc * 0.125f);
}

// Adjoint of the pooling: g[child][off + ch] += gy[parent][ch] / 8 (FP32).
__global__ void k_avgpool_bwd_add(const float* __restrict__ gy, int c, int n, int d, int h, int w, float* __restrict__ g,
                                  int ld, int off) {
    // one thread per fine voxel and four channels; 32-bit indices
    const uint32_t c4 = (uint32_t)c >> 2;
    const uint32_t total = (uint32_t)n * d * h * w * c4;
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    uint32_t r = idx;
    const uint32_t q4 = r % c4; r /= c4;
    const uint32_t x = r % (uint32_t)w; r /= (uint32_t)w;
    const uint32_t y = r % (uint32_t)h; r /= (uint32_t)h;
    const uint32_t z = r % (uint32_t)d;
    const uint32_t s = r / (uint32_t)d;
    const uint32_t p = ((s * (d / 2) + z / 2) * (h / 2) + y / 2) * (w / 2) + x / 2;
    const uint32_t v = ((s * d + z) * h + y) * w + x;
    const float4 t = *(const float4*)(gy + (int64_t)p * c + 4 * q4);
    float4* dst = (float4*)(g + (int64_t)v * ld + off + 4 * q4);
    float4 o = *dst;
    o.x += 0.125f * t.x, o.y += 0.125f * t.y, o.z += 0.125f * t.z, o.w += 0.125f * t.w;
    *dst = o;
}

// Nearest 2x upsampling of BF16 [V][c] (coarse dims d, h, w) into packed
// [8V][c]; c a multiple of 8, copied in 16-byte pieces.
__global__ void k_upsample_fwd(const uint16_t* __restrict__ x, int c, int n, int d, int h, int w,
                               uint16_t* __restrict__ y) {
    const uint32_t D = 2 * d, H = 2 * h, W = 2 * w;
    const uint32_t c8 = (uint32_t)c / 8;
    const uint32_t total = (uint32_t)n * D * H * W * c8;
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    uint32_t r = idx;
    const uint32_t part = r % c8; r /= c8;
    const uint32_t X = r % W; r /= W;
    const uint32_t Y = r % H; r /= H;
    const uint32_t Z = r % D;
    const uint32_t s = r / D;
    const uint32_t p = ((s * d + Z / 2) * h + Y / 2) * w + X / 2;
    ((uint4*)y)[idx] = ((const uint4*)x)[(int64_t)p * c8 + part];
}

// Adjoint of the upsampling: g[parent][ch] = sum of the 8 children (FP32, packed).
__global__ void k_upsample_bwd(const float* __restrict__ gy, int c, int n, int d, int h, int w, float* __restrict__ g) {
    // one thread per coarse voxel and four channels; 32-bit indices (the host
    // checks the sizes)
    const uint32_t c4 = (uint32_t)c >> 2;
    const uint32_t total = (uint32_t)n * d * h * w * c4;
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    uint32_t r = idx;
    const uint32_t q4 = r % c4; r /= c4;
    const uint32_t x = r % (uint32_t)w; r /= (uint32_t)w;
    const uint32_t y = r % (uint32_t)h; r /= (uint32_t)h;
    const uint32_t z = r % (uint32_t)d;
    const uint32_t s = r / (uint32_t)d;
    const uint32_t H = 2 * h, W = 2 * w;
    float4 acc = float4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const uint32_t v = ((s * 2 * d + 2 * z + (k >> 2)) * H + 2 * y + ((k >> 1) & 1)) * W + 2 * x + (k & 1);
        const float4 t = *(const float4*)(gy + (int64_t)v * c + 4 * q4);
        acc.x += t.x, acc.y += t.y, acc.z += t.z, acc.w += t.w;
    }
    *(float4*)(g + (int64_t)idx * 4) = acc;
}

// Fixed trilinear upsampling of channels 0..2 of the FP32 coarse input (row 4):
// fine node 2i on coarse node i, odd nodes average their neighbours, the last
// coarse node repeated.  Output FP32 [8V][ldo], ldo 3 or 4 (channel 3 zero).
__global__ void k_trilinear(const float* __restrict__ x, int n, int d, int h, int w, float* __restrict__ y, int ldo) {
    const int D = 2 * d, H = 2 * h, W = 2 * w;
    const int64_t total = (int64_t)n * D * H * W;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    int64_t r = idx;
    const int X = (int)(r % W); r /= W;
    const int Y = (int)(r % H); r /= H;
    const int Z = (int)(r % D);
    const int s = (int)(r / D);
    const int z0 = Z / 2, y0 = Y / 2, x0 = X / 2;
    const int z1 = (Z & 1) ? (z0 + 1 < d ? z0 + 1 : d - 1) : z0;
    const int y1 = (Y & 1) ? (y0 + 1 < h ? y0 + 1 : h - 1) : y0;
    const int x1 = (X & 1) ? (x0 + 1 < w ? x0 + 1 : w - 1) : x0;
    for (int c = 0; c < 3; ++c) {
        auto at = [&](int zz, int yy, int xx) { return x[((((int64_t)s * d + zz) * h + yy) * w + xx) * 4 + c]; };
        const float v = 0.125f * (at(z0, y0, x0) + at(z0, y0, x1) + at(z0, y1, x0) + at(z0, y1, x1) +
                                  at(z1, y0, x0) + at(z1, y0, x1) + at(z1, y1, x0) + at(z1, y1, x1));
        y[idx * ldo + c] = v;
    }
    if (ldo == 4) y[idx * 4 + 3] = 0.0f;
}

// out[v][c] = base[v][c] + r[v][c], c < 3 (rows: base and r 4, out 3).
__global__ void k_add_residual(const float* __restrict__ base, const float* __restrict__ r, int64_t total,
                               float* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total * 3) return;
    const int64_t v = idx / 3;
    const int c = (int)(idx - v * 3);
    out[idx] = base[v * 4 + c] + r[v * 4 + c];
}

// Masked squared error: per-block partial sums of the mask count and of the
// squared error (FP64), then the gradient dr = 2 (pred - target) mask / (3 count).
__global__ void k_loss_partial(const float* __restrict__ base, const float* __restrict__ r,
                               const float* __restrict__ target, const uint8_t* __restrict__ mask, int64_t total,
                               double* __restrict__ part) {
    __shared__ double s_cnt[256], s_err[256];
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double cnt = 0.0, err = 0.0;
    if (v < total && mask[v]) {
        cnt = 1.0;
        for (int c = 0; c < 3; ++c) {
            const double d = (double)(base[v * 4 + c] + r[v * 4 + c]) - (double)target[v * 3 + c];
            err += d * d;
        }
    }
    s_cnt[threadIdx.x] = cnt;
    s_err[threadIdx.x] = err;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            s_cnt[threadIdx.x] += s_cnt[threadIdx.x + st];
            s_err[threadIdx.x] += s_err[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s_cnt[0];
        part[2 * blockIdx.x + 1] = s_err[0];
    }
}
__global__ void k_loss_reduce(const double* __restrict__ part, int nb, double* __restrict__ out) {
    __shared__ double s_cnt[256], s_err[256];
    double cnt = 0.0, err = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) {
        cnt += part[2 * b];
        err += part[2 * b + 1];
    }
    s_cnt[threadIdx.x] = cnt;
    s_err[threadIdx.x] = err;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            s_cnt[threadIdx.x] += s_cnt[threadIdx.x + st];
            s_err[threadIdx.x] += s_err[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n = s_cnt[0] * 3.0 > 1.0 ? s_cnt[0] * 3.0 : 1.0;
        out[0] = s_err[0] / n;   // loss
        out[1] = n;              // normalisation
    }
}
__global__ void k_loss_grad(const float* __restrict__ base, const float* __restrict__ r,
                            const float* __restrict__ target, const uint8_t* __restrict__ mask, int64_t total,
                            const double* __restrict__ stats, float* __restrict__ dr) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= total) return;
    const float scale = (float)(2.0 / stats[1]);
    for (int c = 0; c < 3; ++c) {
        const float d = mask[v] ? (base[v * 4 + c] + r[v * 4 + c]) - target[v * 3 + c] : 0.0f;
        dr[v * 4 + c] = scale * d;
    }
    dr[v * 4 + 3] = 0.0f;
}

// Adam (Kingma & Ba) on FP32 parameters: m, v moments, bias-corrected step.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t count, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Crops of a batch: coarse input (u, mask) and fine target (u, mask) around
// per-sample coarse origins; zero outside the source fields.  The fine loss
// mask excludes a margin next to the crop faces.
__global__ void k_crop(const float* __restrict__ uc, const uint8_t* __restrict__ mc, int Dc, int Hc, int Wc,
                       const float* __restrict__ uf, const uint8_t* __restrict__ mf, const int* __restrict__ origin,
                       int n, int d, int h, int w, int margin, float* __restrict__ xin, float* __restrict__ tgt,
                       uint8_t* __restrict__ tmask) {
    // 32-bit indices: the host checks that the fine crops and the source
    // grids stay below 2^31 values
    const uint32_t Vc = (uint32_t)d * h * w, Vf = 8 * Vc;
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < (uint32_t)n * Vc) {
        const uint32_t s = idx / Vc;
        const uint32_t r = idx - s * Vc;
        const int x = (int)(r % (uint32_t)w), y = (int)((r / (uint32_t)w) % (uint32_t)h), z = (int)(r / ((uint32_t)w * h));
        const int Z = origin[3 * s] + z, Y = origin[3 * s + 1] + y, X = origin[3 * s + 2] + x;
        const bool in = Z >= 0 && Z < Dc && Y >= 0 && Y < Hc && X >= 0 && X < Wc;
        const uint32_t src = in ? ((uint32_t)Z * Hc + Y) * Wc + X : 0;
        for (int c = 0; c < 3; ++c) xin[(int64_t)idx * 4 + c] = in ? uc[(int64_t)src * 3 + c] : 0.0f;
        xin[(int64_t)idx * 4 + 3] = in ? (float)mc[src] : 0.0f;
    }
    if (idx < (uint32_t)n * Vf) {
        const uint32_t s = idx / Vf;
        const uint32_t r = idx - s * Vf;
        const uint32_t W2 = 2 * w, H2 = 2 * h;
        const int D2 = 2 * d;
        const int x = (int)(r % W2), y = (int)((r / W2) % H2), z = (int)(r / (W2 * H2));
        const int Z = 2 * origin[3 * s] + z, Y = 2 * origin[3 * s + 1] + y, X = 2 * origin[3 * s + 2] + x;
        const int Df = 2 * Dc, Hf = 2 * Hc, Wf = 2 * Wc;
        const bool in = Z >= 0 && Z < Df && Y >= 0 && Y < Hf && X >= 0 && X < Wf;
        const uint32_t src = in ? ((uint32_t)Z * Hf + Y) * Wf + X : 0;
        for (int c = 0; c < 3; ++c) tgt[(int64_t)idx * 3 + c] = in ? uf[(int64_t)src * 3 + c] : 0.0f;
        const bool inner = z >= margin && z < D2 - margin && y >= margin && y < (int)H2 - margin && x >= margin &&
                           x < (int)W2 - margin;
        tmask[idx] = (in && inner && mf[src]) ? 1 : 0;
    }
}

// Scatter of scaled node values (component-major [3][count], FP64) at node
// coordinates into a dense FP32 [D][H][W][3] field and a node mask.
__global__ void k_scatter(const double* __restrict__ vals, const int32_t* __restrict__ xyz, int64_t count, int D,
                          int H, int W, double scale, float* __restrict__ dense, uint8_t* __restrict__ mask) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    if (x < 0 || x >= W || y < 0 || y >= H || z < 0 || z >= D) return;
    const int64_t v = ((int64_t)z * H + y) * W + x;
    for (int c = 0; c < 3; ++c) dense[v * 3 + c] = (float)(scale * vals[c * count + i]);
    mask[v] = 1;
}

// Gather of a dense FP32 [V][3] field at node coordinates into scaled [3][count] FP64.
__global__ void k_gather(const float* __restrict__ dense, const int32_t* __restrict__ xyz, int64_t count, int D, int H,
                         int W, double scale, double* __restrict__ vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    const bool in = x >= 0 && x < W && y >= 0 && y < H && z >= 0 && z < D;
    const int64_t v = in ? ((int64_t)z * H + y) * W + x : 0;
    for (int c = 0; c < 3; ++c) vals[c * count + i] = in ? scale * (double)dense[v * 3 + c] : 0.0;
}

__global__ void k_fill(uint32_t* p, int64_t nwords, uint32_t value) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nwords; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = value;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

template <int CIN>
hipError_t conv_lds(const ConvArgs& a, int mt, bool f32out, hipStream_t st) {
    const dim3 grid((unsigned)((int64_t)a.n * (a.d / BZ) * (a.h / BY) * (a.w / BX))), block(256);
    if (mt == 1 && f32out) hipLaunchKernelGGL((k_conv_fwd_lds<CIN, 1, true>), grid, block, 0, st, a);
    else if (mt == 1) hipLaunchKernelGGL((k_conv_fwd_lds<CIN, 1, false>), grid, block, 0, st, a);
    else if (mt == 2 && f32out) hipLaunchKernelGGL((k_conv_fwd_lds<CIN, 2, true>), grid, block, 0, st, a);
    else if (mt == 2) hipLaunchKernelGGL((k_conv_fwd_lds<CIN, 2, false>), grid, block, 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t conv_forward(const ConvArgs& a, int mt, bool f32out, hipStream_t st) {
    // the brick kernel when the grid tiles into bricks and the staging loads
    // stay aligned (16-byte pieces: row and channel offset multiples of 8
    // channels; 8-byte pieces for 4 channels)
    const bool bricks = a.d % BZ == 0 && a.h % BY == 0 && a.w % BX == 0 && a.kpad == (27 * a.cin + 15) / 16 * 16;
    if (bricks && a.cin == 16 && a.ldx % 8 == 0 && a.cxo % 8 == 0) return conv_lds<16>(a, mt, f32out, st);
    if (bricks && a.cin == 32 && a.ldx % 8 == 0 && a.cxo % 8 == 0) return conv_lds<32>(a, mt, f32out, st);
    if (bricks && a.cin == 4 && a.ldx % 4 == 0 && a.cxo % 4 == 0) return conv_lds<4>(a, mt, f32out, st);
    const int64_t total = (int64_t)a.n * a.d * a.h * a.w;
    const unsigned grid = blocks_for(total, CONV_WAVES * CONV_VOX);
    const dim3 block(CONV_WAVES * 64);
    if (mt == 1 && f32out) hipLaunchKernelGGL((k_conv_fwd<1, true>), dim3(grid), block, 0, st, a);
    else if (mt == 1) hipLaunchKernelGGL((k_conv_fwd<1, false>), dim3(grid), block, 0, st, a);
    else if (mt == 2 && f32out) hipLaunchKernelGGL((k_conv_fwd<2, true>), dim3(grid), block, 0, st, a);
    else if (mt == 2) hipLaunchKernelGGL((k_conv_fwd<2, false>), dim3(grid), block, 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

template <int CIN>
hipError_t wgrad_lds(const WgradArgs& a, int mt, int nparts, hipStream_t st) {
    const int ntiles = a.npad / 16;
    const dim3 grid(nparts, (ntiles + 4 * WG_TPW - 1) / (4 * WG_TPW));
    if (mt == 1) hipLaunchKernelGGL((k_conv_wgrad_lds<CIN, 1>), grid, dim3(256), 0, st, a, nparts);
    else if (mt == 2) hipLaunchKernelGGL((k_conv_wgrad_lds<CIN, 2>), grid, dim3(256), 0, st, a, nparts);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t conv_wgrad(const WgradArgs& a, int mt, int nchunks, int cout_param, float* dw, hipStream_t st,
                      const BiasJob* bias) {
    const int ntiles = a.npad / 16;
    // brick kernel: same tiling and alignment conditions as the forward one;
    // at most nchunks partials (the size the caller's partial buffer holds)
    const bool bricks = a.d % BZ == 0 && a.h % BY == 0 && a.w % BX == 0 && a.npad == (27 * a.cin + 15) / 16 * 16 &&
                        a.cout <= 16 * mt && a.cout % 4 == 0 && a.ldy % 4 == 0 && ((uintptr_t)a.dy & 7) == 0;
    const int64_t nbricks = (int64_t)a.n * (a.d / BZ) * (a.h / BY) * (a.w / BX);
    const int nparts = (int)(nbricks < nchunks ? nbricks : nchunks);
    hipError_t e;
    int nred = nparts;   // partials the reduction sums
    if (bricks && (mt == 1 || mt == 2) && a.mpad >= 16 * mt && a.cin % 16 == 0 && a.cin <= 32 && a.ldx % 8 == 0 &&
        a.cxo % 8 == 0) {
        const dim3 grid(nparts, a.cin / 16 * mt);   // (input group, output group) pairs
        if (a.cin == 16) hipLaunchKernelGGL(k_conv_wgrad_k16<16>, grid, dim3(256), 0, st, a, nparts);
        else hipLaunchKernelGGL(k_conv_wgrad_k16<32>, grid, dim3(256), 0, st, a, nparts);
        e = hipGetLastError();
    } else if (bricks && a.cin == 4 && a.ldx % 4 == 0 && a.cxo % 4 == 0) {
        e = wgrad_lds<4>(a, mt, nparts, st);
    } else {
        const dim3 grid(nchunks, (ntiles + 15) / 16);
        if (mt == 1) hipLaunchKernelGGL((k_conv_wgrad<1>), grid, dim3(256), 0, st, a);
        else if (mt == 2) hipLaunchKernelGGL((k_conv_wgrad<2>), grid, dim3(256), 0, st, a);
        else return hipErrorInvalidValue;
        e = hipGetLastError();
        nred = nchunks;
    }
    if (e != hipSuccess) return e;
    const int N = 27 * a.cin;
    const int wblocks = (int)blocks_for((int64_t)cout_param * N, 32);
    const int bblocks = bias ? bias->cout_param : 0;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(wblocks + bblocks), dim3(256), 0, st, a.part, nred, a.mpad, a.npad,
                       cout_param, N, dw, wblocks, bias ? bias->part : nullptr, bias ? bias->nparts : 0,
                       bias ? bias->db : nullptr);
    return hipGetLastError();
}

hipError_t prep_weights_all(const PrepJobs& jobs, hipStream_t st) {
    if (jobs.n < 1 || jobs.n > MAX_PREP_JOBS) return hipErrorInvalidValue;
    int64_t n = 0;
    for (int i = 0; i < jobs.n; ++i) {
        const PrepJob& p = jobs.j[i];
        const int64_t a = (int64_t)p.mpad * p.kpad, b = p.wd ? (int64_t)p.mpad_d * p.kpad_d : 0;
        n = a > n ? a : n;
        n = b > n ? b : n;
    }
    hipLaunchKernelGGL(k_prep_weights_all, dim3(blocks_for(n, 256), jobs.n), dim3(256), 0, st, jobs);
    return hipGetLastError();
}

hipError_t prep_weights(const float* w, int cin, int cout_param, int cout, uint16_t* wt, int mpad, int kpad,
                        uint16_t* wd, int mpad_d, int kpad_d, hipStream_t st) {
    int64_t n = (int64_t)mpad * kpad;
    if (wd && (int64_t)mpad_d * kpad_d > n) n = (int64_t)mpad_d * kpad_d;
    hipLaunchKernelGGL(k_prep_weights, dim3(blocks_for(n, 256)), dim3(256), 0, st, w, cin, cout_param, cout, wt, mpad,
                       kpad, wd, mpad_d, kpad_d);
    return hipGetLastError();
}

hipError_t grad_relu_cast(const float* g, int ldg, int offg, const uint16_t* act, int lda, int offa, int c,
                          int64_t total, uint16_t* out, float* part, int cout_param, float* db, hipStream_t st,
                          BiasJob* defer) {
    // c channels of partial sums per work-group fit the 64-float rows of part
    if (c <= 0 || c > 64 || 256 % c != 0 || cout_param > c) return hipErrorInvalidValue;
    const bool vec = c % 4 == 0 && ldg % 4 == 0 && offg % 4 == 0 && ((uintptr_t)g & 15) == 0 &&
                     ((uintptr_t)out & 7) == 0 && (!act || (lda % 4 == 0 && offa % 4 == 0 && ((uintptr_t)act & 7) == 0));
    const int64_t align = vec ? 1024 : 256;   // elements per work-group: a multiple of this
    const int64_t E = total * c;
    int64_t nb = (E + 4095) / 4096;
    if (nb > BIAS_PARTS) nb = BIAS_PARTS;
    if (nb < 1) nb = 1;
    const int64_t per = ((E + nb - 1) / nb + align - 1) / align * align;
    nb = (E + per - 1) / per;
    if (nb < 1) nb = 1;
    if (vec)
        hipLaunchKernelGGL(k_grad_relu_cast4, dim3((unsigned)nb), dim3(256), 0, st, g, ldg, offg, act, lda, offa, c,
                           total, per, out, part);
    else
        hipLaunchKernelGGL(k_grad_relu_cast, dim3((unsigned)nb), dim3(256), 0, st, g, ldg, offg, act, lda, offa, c,
                           total, per, out, part);
    if (defer) {   // the caller reduces the partials later (conv_wgrad of the same layer)
        *defer = BiasJob{part, (int)nb, cout_param, db};
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_bias_reduce, dim3(cout_param), dim3(256), 0, st, part, (int)nb, db);
    return hipGetLastError();
}

hipError_t cast_input(const float* x, int64_t count, uint16_t* out, hipStream_t st) {
    hipLaunchKernelGGL(k_cast_input, dim3(blocks_for(count, 256)), dim3(256), 0, st, x, count, out);
    return hipGetLastError();
}

hipError_t avgpool_fwd(const uint16_t* x, int ld, int off, int c, int n, int d, int h, int w, uint16_t* y,
                       hipStream_t st) {
    const int64_t total = (int64_t)n * (d / 2) * (h / 2) * (w / 2) * c;
    hipLaunchKernelGGL(k_avgpool_fwd, dim3(blocks_for(total, 256)), dim3(256), 0, st, x, ld, off, c, n, d, h, w, y);
    return hipGetLastError();
}

hipError_t avgpool_bwd_add(const float* gy, int c, int n, int d, int h, int w, float* g, int ld, int off,
                           hipStream_t st) {
    // four channels per thread, 16-byte aligned rows, 32-bit voxel indices
    const int64_t vox = (int64_t)n * d * h * w;
    if (c % 4 != 0 || ld % 4 != 0 || off % 4 != 0 || ((uintptr_t)g & 15) || ((uintptr_t)gy & 15) ||
        vox * (ld > c ? ld : c) >= ((int64_t)1 << 31))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_avgpool_bwd_add, dim3(blocks_for(vox * (c / 4), 256)), dim3(256), 0, st, gy, c, n, d, h, w, g,
                       ld, off);
    return hipGetLastError();
}

hipError_t upsample_fwd(const uint16_t* x, int c, int n, int d, int h, int w, uint16_t* y, hipStream_t st) {
    const int64_t total = (int64_t)n * 8 * d * h * w * (c / 8);
    if (c % 8 != 0 || total * 8 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_upsample_fwd, dim3(blocks_for(total, 256)), dim3(256), 0, st, x, c, n, d, h, w, y);
    return hipGetLastError();
}

hipError_t upsample_bwd(const float* gy, int c, int n, int d, int h, int w, float* g, hipStream_t st) {
    // four channels per thread, 32-bit indices over the fine grid
    const int64_t vox = (int64_t)n * d * h * w;
    if (c % 4 != 0 || ((uintptr_t)g & 15) || ((uintptr_t)gy & 15) || vox * 8 * c >= ((int64_t)1 << 31))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_upsample_bwd, dim3(blocks_for(vox * (c / 4), 256)), dim3(256), 0, st, gy, c, n, d, h, w, g);
    return hipGetLastError();
}

hipError_t trilinear(const float* x, int n, int d, int h, int w, float* y, int ldo, hipStream_t st) {
    const int64_t total = (int64_t)n * 8 * d * h * w;
    hipLaunchKernelGGL(k_trilinear, dim3(blocks_for(total, 256)), dim3(256), 0, st, x, n, d, h, w, y, ldo);
    return hipGetLastError();
}

hipError_t add_residual(const float* base, const float* r, int64_t total, float* out, hipStream_t st) {
    hipLaunchKernelGGL(k_add_residual, dim3(blocks_for(total * 3, 256)), dim3(256), 0, st, base, r, total, out);
    return hipGetLastError();
}

hipError_t loss_and_grad(const float* base, const float* r, const float* target, const uint8_t* mask, int64_t total,
                         double* part, double* stats, float* dr, hipStream_t st) {
    const unsigned nb = blocks_for(total, 256);
    hipLaunchKernelGGL(k_loss_partial, dim3(nb), dim3(256), 0, st, base, r, target, mask, total, part);
    hipLaunchKernelGGL(k_loss_reduce, dim3(1), dim3(256), 0, st, part, (int)nb, stats);
    if (dr) hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(256), 0, st, base, r, target, mask, total, stats, dr);
    return hipGetLastError();
}

hipError_t adam(float* w, const float* g, float* m, float* v, int64_t count, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(count, 256)), dim3(256), 0, st, w, g, m, v, count, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

hipError_t crop(const float* uc, const uint8_t* mc, int Dc, int Hc, int Wc, const float* uf, const uint8_t* mf,
                const int* origin, int n, int d, int h, int w, int margin, float* xin, float* tgt, uint8_t* tmask,
                hipStream_t st) {
    const int64_t total = (int64_t)n * 8 * d * h * w;
    if (total >= ((int64_t)1 << 31) || (int64_t)8 * Dc * Hc * Wc >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_crop, dim3(blocks_for(total, 256)), dim3(256), 0, st, uc, mc, Dc, Hc, Wc, uf, mf, origin, n,
                       d, h, w, margin, xin, tgt, tmask);
    return hipGetLastError();
}

hipError_t scatter(const double* vals, const int32_t* xyz, int64_t count, int D, int H, int W, double scale,
                   float* dense, uint8_t* mask, hipStream_t st) {
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(count, 256)), dim3(256), 0, st, vals, xyz, count, D, H, W, scale,
                       dense, mask);
    return hipGetLastError();
}

hipError_t gather(const float* dense, const int32_t* xyz, int64_t count, int D, int H, int W, double scale,
                  double* vals, hipStream_t st) {
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(count, 256)), dim3(256), 0, st, dense, xyz, count, D, H, W, scale,
                       vals);
    return hipGetLastError();
}

hipError_t fill(void* p, size_t bytes, uint32_t value, hipStream_t st) {
    const int64_t nw = (int64_t)(bytes / 4);
    if (nw == 0) return hipSuccess;
    unsigned blocks = blocks_for(nw, 256);
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, st, (uint32_t*)p, nw, value);
    return hipGetLastError();
}

}  // namespace lbmnet_dev
