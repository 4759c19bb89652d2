// Batched stepping of many domains (gfx950): every launch covers the blocks of
// all domains of a batch, so small and uneven geometries fill the device
// together instead of one after another.  Two forms:
//  - k_batch_step: one launch per step (captured K at a time into a graph);
//  - k_batch_persistent: one launch for K steps; the work-groups loop over the
//    work items and meet at a device-wide barrier between steps.
// Both call the same per-block step as the single-domain kernel, so each
// domain's populations are bit-identical to stepping it alone.  Per-step
// launches also stream in place: every domain of the group holds one buffer
// in the same in-place layout, and the host names the kind of each launch.
#include "lbm_device.h"

#include <type_traits>

namespace lbm {
namespace {

// Bound of a barrier wait (iterations of a ~100-cycle sleep, about 0.2 s).
constexpr unsigned SPIN_LIMIT = 1u << 21;

template <class S, bool MON, bool ONE, bool NT, int BS, bool CUR, int IP = STREAM_PULL>
__device__ __forceinline__ void batch_item(const BatchArgs& b, int item, int step) {
    const int packed = b.item_map[item];
    StepArgs a = b.doms[packed >> ITEM_DOMAIN_SHIFT];
    // odd steps: the other time slot (pull: and the other buffer; in place
    // the two pointers are the same buffer)
    if (step & 1) {
        const void* t = a.fin;
        a.fin = a.fout;
        a.fout = const_cast<void*>(t);
        a.tin ^= 1;
    }
    const int lb = packed & ITEM_BLOCK_MASK;
    // ONE: every domain of the batch is CHM-MRT with free rates of one.
    // Otherwise each item takes its own domain's collision form, as the
    // domain's own step would (the forms round differently).
    const bool one = ONE || (a.collision == 0 && a.s[1] == 1.0 && a.s[2] == 1.0 && a.s[3] == 1.0 && a.s[4] == 1.0);
    if (one) {
        if (a.periodic & 6) step_block<S, MON, 1, true, NT, BS, CUR, IP>(a, lb);
        else step_block<S, MON, 1, false, NT, BS, CUR, IP>(a, lb);
    } else if (a.collision == 1) {
        if (a.periodic & 6) step_block<S, MON, 2, true, NT, BS, CUR, IP>(a, lb);
        else step_block<S, MON, 2, false, NT, BS, CUR, IP>(a, lb);
    } else {
        if (a.periodic & 6) step_block<S, MON, 0, true, NT, BS, CUR, IP>(a, lb);
        else step_block<S, MON, 0, false, NT, BS, CUR, IP>(a, lb);
    }
}

template <class S, bool MON, bool ONE, bool NT, int BS, bool CUR, int IP = STREAM_PULL>
__global__ __launch_bounds__(BS) void k_batch_step(BatchArgs b, int step) {
    // XCD-aware order as in the single-domain kernel
    const int hb = blockIdx.x;
    const int item = (hb & 7) * b.items_per_xcd + (hb >> 3);
    if (item >= b.nitems) return;
    batch_item<S, MON, ONE, NT, BS, CUR, IP>(b, item, step);
}

// Device-wide barrier for epoch e (1, 2, ... within one launch; the host clears
// the barrier words before every persistent launch).  Work-group g publishes
// its arrival in its own word (no contention); work-group 0 waits for every
// arrival, then publishes the release; the others wait for the release.
// Every wait is bounded: on a timeout the error flag is set and every
// work-group leaves.  Layout: barrier[0] release epoch, barrier[64 + g] arrival
// of work-group g (at most MAX_PERSISTENT_GROUPS).
__device__ bool grid_barrier(const BatchArgs& b, unsigned epoch) {
    __shared__ int bad;
    unsigned* release = b.barrier;
    unsigned* arrive = b.barrier + 64;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();   // this work-group's stores happen before its arrival
        __hip_atomic_store(arrive + blockIdx.x, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (blockIdx.x == 0) {
        for (unsigned k = threadIdx.x; k < gridDim.x && !bad; k += blockDim.x) {
            unsigned spins = 0;
            while (__hip_atomic_load(arrive + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > SPIN_LIMIT || __hip_atomic_load(b.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                    bad = 1;
                    break;
                }
            }
        }
        __threadfence();   // the observed work-groups' stores happen before the release
        __syncthreads();
        if (threadIdx.x == 0) {
            if (bad) atomicExch(b.error, 1);
            __threadfence();
            __hip_atomic_store(release, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (threadIdx.x == 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(release, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > SPIN_LIMIT || __hip_atomic_load(b.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                atomicExch(b.error, 1);
                bad = 1;
                break;
            }
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();   // acquire the other work-groups' stores
        if (__hip_atomic_load(b.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) bad = 1;
    }
    __syncthreads();
    return bad == 0;
}

// Steps step0 .. step0 + nsteps - 1 without monitors (the monitored last step
// of a sequence is a k_batch_step launch).
template <class S, bool ONE, bool NT, int BS, bool CUR>
__global__ __launch_bounds__(BS) void k_batch_persistent(BatchArgs b, int step0, int nsteps) {
    for (int s = 0; s < nsteps; ++s) {
        for (int item = blockIdx.x; item < b.nitems; item += gridDim.x)
            batch_item<S, false, ONE, NT, BS, CUR>(b, item, step0 + s);
        if (s + 1 < nsteps && !grid_barrier(b, (unsigned)(s + 1))) return;
    }
}

// FP32 with streaming stores caps the resident work-groups of 256 threads at
// six per CU through the dynamic LDS size, as the single-domain step does
// (6 x 26000 B fits the CU's 160 KiB, 7 x does not).
constexpr unsigned BATCH_LDS_SIX_PER_CU = 26000;

template <class S, bool ONE, bool NT, int BS, bool CUR, int IP = STREAM_PULL>
hipError_t step_bs(const BatchArgs& b, int step, bool monitor, hipStream_t st) {
    const dim3 grid(8 * b.items_per_xcd), block(BS);
    const unsigned lds = (NT && sizeof(S) == 4 && BS == 256) ? BATCH_LDS_SIX_PER_CU : 0u;
    if (monitor) hipLaunchKernelGGL((k_batch_step<S, true, ONE, NT, BS, CUR, IP>), grid, block, lds, st, b, step);
    else hipLaunchKernelGGL((k_batch_step<S, false, ONE, NT, BS, CUR, IP>), grid, block, lds, st, b, step);
    return hipGetLastError();
}

// In-place launches: 256 threads, cached stores, no curved-wall blend.
template <class S, bool ONE>
hipError_t step_inplace_one(int kind, const BatchArgs& b, int step, bool monitor, hipStream_t st) {
    if (kind & BATCH_IP_LOCAL) return step_bs<S, ONE, false, 256, false, STREAM_LOCAL>(b, step, monitor, st);
    return step_bs<S, ONE, false, 256, false, STREAM_NEIGHBOUR>(b, step, monitor, st);
}

template <class S, bool ONE, bool NT, int BS, bool CUR>
hipError_t persistent_bs(const BatchArgs& b, int grid, int step0, int nsteps, hipStream_t st) {
    hipLaunchKernelGGL((k_batch_persistent<S, ONE, NT, BS, CUR>), dim3(grid), dim3(BS), 0, st, b, step0, nsteps);
    return hipGetLastError();
}

template <class S, bool ONE, bool NT, int BS, bool CUR>
hipError_t capacity_bs(int* blocks) {
    int per_cu = 0, dev = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_persistent<S, ONE, NT, BS, CUR>, BS, 0);
    if (e != hipSuccess) return e;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    *blocks = per_cu * cus;
    return hipSuccess;
}

// Dispatch over (kind, stream_store, block); F is called as F<S, ONE, NT, BS, CUR>().
#define BATCH_BS(S, ONE, NT, CUR, F, ...)                                         \
    switch (c.block) {                                                            \
        case 128: return F<S, ONE, NT, 128, CUR>(__VA_ARGS__);                    \
        case 256: return F<S, ONE, NT, 256, CUR>(__VA_ARGS__);                    \
        case 512: return F<S, ONE, NT, 512, CUR>(__VA_ARGS__);                    \
        default: return hipErrorInvalidValue;                                     \
    }
#define BATCH_NT(S, ONE, CUR, F, ...)                                             \
    if constexpr (sizeof(S) >= 4) {                                               \
        if (c.stream_store) BATCH_BS(S, ONE, true, CUR, F, __VA_ARGS__)          \
    }                                                                             \
    BATCH_BS(S, ONE, false, CUR, F, __VA_ARGS__)

template <class S, bool ONE, bool CUR>
hipError_t step_one(const BatchArgs& b, const BatchConfig& c, int step, bool monitor, hipStream_t st) {
    BATCH_NT(S, ONE, CUR, step_bs, b, step, monitor, st)
}

template <class S, bool ONE, bool CUR>
hipError_t persistent_one(const BatchArgs& b, const BatchConfig& c, int grid, int step0, int nsteps, hipStream_t st) {
    BATCH_NT(S, ONE, CUR, persistent_bs, b, grid, step0, nsteps, st)
}

template <class S, bool ONE, bool CUR>
hipError_t capacity_one(const BatchConfig& c, int* blocks) {
    BATCH_NT(S, ONE, CUR, capacity_bs, blocks)
}

// F<S, ONE, CUR>(args...) for the two flags of kind
#define BATCH_KIND(F, ...)                                                                         \
    switch (kind & (BATCH_RATES_ONE | BATCH_CURVED)) {                                             \
        case 0: return F<S, false, false>(__VA_ARGS__);                                            \
        case BATCH_RATES_ONE: return F<S, true, false>(__VA_ARGS__);                               \
        case BATCH_CURVED: return F<S, false, true>(__VA_ARGS__);                                  \
        default: return F<S, true, true>(__VA_ARGS__);                                             \
    }

template <class S>
hipError_t step_s(int kind, const BatchArgs& b, const BatchConfig& c, int step, bool monitor, hipStream_t st) {
    if (kind & (BATCH_IP_NEIGHBOUR | BATCH_IP_LOCAL)) {
        if (c.mode != BATCH_MODE_INPLACE || c.block != 256 || c.stream_store || (kind & BATCH_CURVED))
            return hipErrorInvalidValue;
        return (kind & BATCH_RATES_ONE) ? step_inplace_one<S, true>(kind, b, step, monitor, st)
                                        : step_inplace_one<S, false>(kind, b, step, monitor, st);
    }
    BATCH_KIND(step_one, b, c, step, monitor, st)
}

template <class S>
hipError_t capacity_s(int kind, const BatchConfig& c, int* blocks) {
    BATCH_KIND(capacity_one, c, blocks)
}

template <class S>
hipError_t persistent_s(int kind, const BatchArgs& b, const BatchConfig& c, int step0, int nsteps, hipStream_t st) {
    int grid = c.grid;
    int cap = 0;
    hipError_t e = capacity_s<S>(kind, c, &cap);
    if (e != hipSuccess) return e;
    // never more work-groups than fit at once: the barrier needs them all resident
    if (grid <= 0 || grid > cap) grid = cap;
    if (grid > b.nitems) grid = b.nitems;
    if (grid > MAX_PERSISTENT_GROUPS) grid = MAX_PERSISTENT_GROUPS;
    BATCH_KIND(persistent_one, b, c, grid, step0, nsteps, st)
}

}  // namespace

// One storage type per translation unit (LBM_BATCH_STORAGE = 0 f64, 1 f32,
// 2 f16s, 3 bf16s), so the four instantiations compile in parallel.
#if !defined(LBM_BATCH_STORAGE)
#error "compile with -DLBM_BATCH_STORAGE=0..3"
#elif LBM_BATCH_STORAGE == 0
#define LBM_BATCH_T double
#elif LBM_BATCH_STORAGE == 1
#define LBM_BATCH_T float
#elif LBM_BATCH_STORAGE == 2
#define LBM_BATCH_T _Float16
#else
#define LBM_BATCH_T __bf16
#endif

hipError_t launch_batch_step_s(int storage, int kind, const BatchArgs& b, const BatchConfig& c, int step,
                               bool monitor, hipStream_t stream, std::integral_constant<int, LBM_BATCH_STORAGE>) {
    (void)storage;
    return step_s<LBM_BATCH_T>(kind, b, c, step, monitor, stream);
}

hipError_t launch_batch_persistent_s(int storage, int kind, const BatchArgs& b, const BatchConfig& c,
                                     int step0, int nsteps, hipStream_t stream,
                                     std::integral_constant<int, LBM_BATCH_STORAGE>) {
    (void)storage;
    return persistent_s<LBM_BATCH_T>(kind, b, c, step0, nsteps, stream);
}

hipError_t batch_persistent_capacity_s(int storage, int kind, const BatchConfig& c, int* blocks,
                                       std::integral_constant<int, LBM_BATCH_STORAGE>) {
    (void)storage;
    return capacity_s<LBM_BATCH_T>(kind, c, blocks);
}

}  // namespace lbm
