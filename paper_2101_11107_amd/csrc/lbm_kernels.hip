// Single-domain HIP kernels of the lattice Boltzmann library (gfx950) and
// their launchers: initialisation, moments, population read-out, monitor
// reduction and buffer clearing (the step kernel is in lbm_step.hip).
#include "lbm_device.h"

namespace lbm {
namespace {

// Initial state: f(0) = f_eq(rho, u), then the first collision (written to
// fout), and the open-link terms for the first step.
template <class S>
__global__ __launch_bounds__(BLOCK) void k_init(StepArgs a, const double* rho0, const double* u0) {
    using T = typename Traits<S>::T;
    constexpr uint32_t SZ = sizeof(S);
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i == 0) {
        a.tcount[0] = 0;
        a.tcount[1] = 0;
    }
    if (i >= a.n) return;
    const double r = rho0 ? rho0[i] : 1.0;
    const double u[3] = {u0 ? u0[i] : 0.0, u0 ? u0[a.n + i] : 0.0, u0 ? u0[2 * a.n + i] : 0.0};
    T f[27];
    // the rest state is exactly zero in shifted variables
#pragma unroll
    for (int al = 0; al < 27; ++al)
        f[al] = (rho0 || u0) ? (T)((a.collision == 1 ? feq2(al, r, u) : feq1(al, r, u)) - wgt(al)) : T(0);
    T ux, uy, uz, drho, jx, jy, jz;
    if (a.collision == 1)
        collide<T, 2>(f, a, ux, uy, uz, drho, jx, jy, jz);
    else if (a.s[1] == 1.0 && a.s[2] == 1.0 && a.s[3] == 1.0 && a.s[4] == 1.0)
        collide<T, 1>(f, a, ux, uy, uz, drho, jx, jy, jz);
    else
        collide<T, 0>(f, a, ux, uy, uz, drho, jx, jy, jz);
    const uint32_t w = a.node[i];
    if (w & SPECIAL_BIT) {
        const LBM_GLOBAL SpecialNode* sp = (const LBM_GLOBAL SpecialNode*)a.spec + (w & ~SPECIAL_BIT);
        if (sp->linkmask != 0u) update_links(a, sp, (double)ux, (double)uy, (double)uz, 0);
    }
    LBM_GLOBAL char* fout = (LBM_GLOBAL char*)a.fout;
#pragma unroll
    for (int al = 0; al < 27; ++al) stp<S>(fout, pop_index((uint32_t)i, (uint32_t)al, (uint32_t)a.npad, SZ) * SZ, f[al]);
}

// rho and u of the current state from the post-collision populations, in FP64:
// rho = 1 + sum f_hat*, u = (sum c f_hat* - rho g / 2) / rho (the collision adds
// rho g to j and keeps rho).  mode 0: write rho/u; 1: avg += u; 2: out = avg / count.
template <class S>
__global__ __launch_bounds__(BLOCK) void k_moments(StepArgs a, double* rho, double* u, double* avg,
                                                  int mode, double count) {
    constexpr uint32_t SZ = sizeof(S);
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= a.n) return;
    const int n = a.n;
    if (mode == 2) {
        const double inv = 1.0 / count;
        u[i] = avg[i] * inv;
        u[n + i] = avg[n + i] * inv;
        u[2 * n + i] = avg[2 * n + i] * inv;
        return;
    }
    const LBM_GLOBAL char* fin = (const LBM_GLOBAL char*)a.fin;
    double d = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int al = 0; al < 27; ++al) {
        const double v = (double)ldp<S>(fin, pop_index((uint32_t)i, (uint32_t)al, (uint32_t)a.npad, SZ) * SZ);
        d += v;
        jx += cxo(al) * v;
        jy += cyo(al) * v;
        jz += czo(al) * v;
    }
    const double r = 1.0 + d;
    const double ux = (jx - 0.5 * r * a.g[0]) / r;
    const double uy = (jy - 0.5 * r * a.g[1]) / r;
    const double uz = (jz - 0.5 * r * a.g[2]) / r;
    if (mode == 0) {
        if (rho) rho[i] = r;
        if (u) {
            u[i] = ux;
            u[n + i] = uy;
            u[2 * n + i] = uz;
        }
    } else {
        avg[i] += ux;
        avg[n + i] += uy;
        avg[2 * n + i] += uz;
    }
}

template <class S>
__global__ __launch_bounds__(BLOCK) void k_read_pop(StepArgs a, double* out) {
    constexpr uint32_t SZ = sizeof(S);
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= a.n) return;
    const LBM_GLOBAL char* fin = (const LBM_GLOBAL char*)a.fin;
#pragma unroll
    for (int al = 0; al < 27; ++al)
        out[(size_t)al * a.n + i] = (double)ldp<S>(fin, pop_index((uint32_t)i, (uint32_t)al, (uint32_t)a.npad, SZ) * SZ);
}

// Fixed-order reduction of the per-block monitor partials (one work-group).
__global__ __launch_bounds__(BLOCK) void k_mon_final(const double* __restrict__ part, int nb,
                                                     double* __restrict__ out) {
    __shared__ double sh[BLOCK][9];
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += BLOCK) {
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] += part[(size_t)b * MON_WORDS + k];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) sh[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int k = 0; k < 9; ++k) sh[threadIdx.x][k] += sh[threadIdx.x + s][k];
        }
        __syncthreads();
    }
    if (threadIdx.x < 9) out[threadIdx.x] = sh[0][threadIdx.x];
}

__global__ void k_fill_zero(uint32_t* p, size_t nwords) {
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < nwords;
         k += (size_t)gridDim.x * blockDim.x)
        p[k] = 0u;
}

template <class S>
hipError_t init_t(const StepArgs& a, const double* rho, const double* u, hipStream_t st) {
    hipLaunchKernelGGL((k_init<S>), dim3((a.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, a, rho, u);
    return hipGetLastError();
}
template <class S>
hipError_t moments_t(const StepArgs& a, double* rho, double* u, double* avg, int mode, double count,
                     hipStream_t st) {
    hipLaunchKernelGGL((k_moments<S>), dim3((a.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, a, rho, u,
                       avg, mode, count);
    return hipGetLastError();
}
template <class S>
hipError_t readpop_t(const StepArgs& a, double* out, hipStream_t st) {
    hipLaunchKernelGGL((k_read_pop<S>), dim3((a.n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, st, a, out);
    return hipGetLastError();
}

}  // namespace

// Storage codes follow lbm.h: 0 F64, 1 F32, 2 F16S, 3 BF16S.
#define LBM_DISPATCH(storage, FN, ...)                                  \
    switch (storage) {                                                  \
        case 0: return FN<double>(__VA_ARGS__);                         \
        case 1: return FN<float>(__VA_ARGS__);                          \
        case 2: return FN<_Float16>(__VA_ARGS__);                       \
        case 3: return FN<__bf16>(__VA_ARGS__);                         \
        default: return hipErrorInvalidValue;                           \
    }

hipError_t launch_step(int storage, const StepArgs& a, StepVariant v, hipStream_t stream) {
    switch (storage) {
        case 0: return launch_step_s(a, v, stream, std::integral_constant<int, 0>());
        case 1: return launch_step_s(a, v, stream, std::integral_constant<int, 1>());
        case 2: return launch_step_s(a, v, stream, std::integral_constant<int, 2>());
        case 3: return launch_step_s(a, v, stream, std::integral_constant<int, 3>());
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_inplace_reverse(int storage, const StepArgs& a, bool fill_side, hipStream_t stream) {
    switch (storage) {
        case 0: return launch_inplace_reverse_s(a, fill_side, stream, std::integral_constant<int, 0>());
        case 1: return launch_inplace_reverse_s(a, fill_side, stream, std::integral_constant<int, 1>());
        case 2: return launch_inplace_reverse_s(a, fill_side, stream, std::integral_constant<int, 2>());
        case 3: return launch_inplace_reverse_s(a, fill_side, stream, std::integral_constant<int, 3>());
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_inplace_unstream(int storage, const StepArgs& a, hipStream_t stream) {
    switch (storage) {
        case 0: return launch_inplace_unstream_s(a, stream, std::integral_constant<int, 0>());
        case 1: return launch_inplace_unstream_s(a, stream, std::integral_constant<int, 1>());
        case 2: return launch_inplace_unstream_s(a, stream, std::integral_constant<int, 2>());
        case 3: return launch_inplace_unstream_s(a, stream, std::integral_constant<int, 3>());
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(int storage, const StepArgs& a, const double* rho, const double* u,
                       hipStream_t stream) {
    LBM_DISPATCH(storage, init_t, a, rho, u, stream);
}

hipError_t launch_moments(int storage, const StepArgs& a, double* rho, double* u, double* avg,
                          int avg_mode, double avg_count, hipStream_t stream) {
    LBM_DISPATCH(storage, moments_t, a, rho, u, avg, avg_mode, avg_count, stream);
}

hipError_t launch_read_populations(int storage, const StepArgs& a, double* out, hipStream_t stream) {
    LBM_DISPATCH(storage, readpop_t, a, out, stream);
}

hipError_t launch_monitor_finalize(const double* partials, int nblocks, double* out,
                                   hipStream_t stream) {
    hipLaunchKernelGGL(k_mon_final, dim3(1), dim3(BLOCK), 0, stream, partials, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t stream) {
    const size_t nw = bytes / 4;
    if (nw == 0) return hipSuccess;
    size_t blocks = (nw + BLOCK - 1) / BLOCK;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(BLOCK), 0, stream, (uint32_t*)p, nw);
    return hipGetLastError();
}

}  // namespace lbm
