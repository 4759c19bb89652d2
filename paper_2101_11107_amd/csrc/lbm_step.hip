// Single-domain step kernel (gfx950) and its launcher, compiled once per
// storage type (LBM_STEP_STORAGE = 0 f64, 1 f32, 2 f16s, 3 bf16s) so the
// variants compile in parallel.
#include "lbm_device.h"

#include <type_traits>

namespace lbm {
namespace {

// One step over one domain.  XCD-aware order: hardware work-group b runs on
// XCD (b % 8); each XCD gets a contiguous range of the node list, so
// neighbouring rows share its L2.
template <class S, bool MON, int FORM, bool PER, bool NT, bool CURVED, int IP = STREAM_PULL>
__global__ __launch_bounds__(BLOCK) void k_step(StepArgs a) {
    const int hb = blockIdx.x;
    const int lb = (hb & 7) * a.blocks_per_xcd + (hb >> 3);
    if (lb >= a.nblocks) return;
    step_block<S, MON, FORM, PER, NT, BLOCK, CURVED, IP>(a, lb);
}

// In-place streaming, pull layout <-> reversed layout: every node swaps its
// slots a and abar (bit copies, no rounding).  FILL (entering from the pull
// layout with curved walls): each wall link's record entry of a.cside takes
// the node's own f*_al(x), in the record order of curved_blend.
template <class S, bool PER, bool FILL>
__global__ __launch_bounds__(BLOCK) void k_inplace_reverse(StepArgs a) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= a.n) return;
    LBM_GLOBAL char* buf = (LBM_GLOBAL char*)a.fin;
    const uint32_t own = node_off<S>((uint32_t)i);
    S v[27];
#pragma unroll
    for (int al = 0; al < 27; ++al) v[al] = *(const LBM_GLOBAL S*)(buf + dir_off(al) + own);
    if (FILL) {
        const uint32_t w = ((const LBM_GLOBAL uint32_t*)a.node)[i];
        uint32_t wallmask = 0, loc[27];
        if (!(w & SPECIAL_BIT)) {
            typename Traits<S>::T unused[27];
            gather_fast<S, PER, true, GATHER_WALL_BITS>(buf, a, i, w, unused, wallmask, loc);
        } else {
            wallmask = ((const LBM_GLOBAL SpecialNode*)a.spec + (w & ~SPECIAL_BIT))->wallmask;
        }
        if (__ballot(wallmask != 0u)) {
            LBM_GLOBAL S* side = (LBM_GLOBAL S*)a.cside;
            const int chunk = __builtin_amdgcn_readfirstlane(i / CREC_CHUNK);
            uint32_t cum = ((const LBM_GLOBAL uint32_t*)a.crec_base)[chunk];
#pragma unroll
            for (int al = 0; al < 27; ++al) {
                if (al == 13) continue;
                const bool wl = (wallmask >> al) & 1u;
                const unsigned long long B = __ballot(wl);
                if (B == 0ull) continue;
                const uint32_t idx =
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(B >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)B, cum));
                cum += (uint32_t)__popcll(B);
                if (wl) side[idx] = v[al];
            }
        }
    }
#pragma unroll
    for (int al = 0; al < 27; ++al) *(LBM_GLOBAL S*)(buf + dir_off(26 - al) + own) = v[al];
}

// In-place streaming, streamed layout (a.fin) -> pull layout (a.fout): the
// neighbour step's reads give f*_abar of this node for every direction al
// (the values are only moved; the storage conversions are exact both ways).
template <class S, bool PER>
__global__ __launch_bounds__(BLOCK) void k_inplace_unstream(StepArgs a) {
    using T = typename Traits<S>::T;
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= a.n) return;
    const LBM_GLOBAL char* fin = (const LBM_GLOBAL char*)a.fin;
    LBM_GLOBAL char* fout = (LBM_GLOBAL char*)a.fout;
    const uint32_t w = ((const LBM_GLOBAL uint32_t*)a.node)[i];
    const uint32_t own = node_off<S>((uint32_t)i);
    T f[27];
    uint32_t loc[27], wallmask = 0;
    if (!(w & SPECIAL_BIT)) {
        gather_fast<S, PER, false, STREAM_NEIGHBOUR>(fin, a, i, w, f, wallmask, loc);
    } else {
        const LBM_GLOBAL SpecialNode* sp = (const LBM_GLOBAL SpecialNode*)a.spec + (w & ~SPECIAL_BIT);
        const uint32_t nonfluid = sp->wallmask | sp->linkmask;
#pragma unroll
        for (int al = 0; al < 27; ++al) f[al] = ldp<S>(fin, inplace_special_off<S>(sp, al, nonfluid, own));
    }
#pragma unroll
    for (int al = 0; al < 27; ++al) stp<S>(fout + dir_off(26 - al), own, f[al]);
}

// FP32 steps of domains beyond the Infinity Cache run six work-groups per CU
// instead of the eight their registers allow: each work-group then lives a
// shorter time, so the tail at the end of a step drains sooner (measured 1 %
// faster at 512^3; the 2-byte forms lose with fewer waves, FP64 is limited to
// five by its registers).  The cap is set through the dynamic LDS size:
// 6 x (26000 B + the monitor's static LDS) fits the CU's 160 KiB, 7 x does not.
constexpr unsigned STEP_LDS_SIX_PER_CU = 26000;

template <class S, bool MON, int FORM, bool NT, bool CURVED, int IP = STREAM_PULL>
hipError_t step_per(const StepArgs& a, bool per, hipStream_t st) {
    const dim3 grid(8 * a.blocks_per_xcd), block(BLOCK);
    const unsigned lds = (NT && sizeof(S) == 4) ? STEP_LDS_SIX_PER_CU : 0u;
    if (per) hipLaunchKernelGGL((k_step<S, MON, FORM, true, NT, CURVED, IP>), grid, block, lds, st, a);
    else hipLaunchKernelGGL((k_step<S, MON, FORM, false, NT, CURVED, IP>), grid, block, lds, st, a);
    return hipGetLastError();
}

// In-place steps keep their stores cached: the next step reads the same
// buffer, which the Infinity Cache can hold where two buffers do not fit.
template <class S, bool MON, int FORM, bool CURVED>
hipError_t step_inplace(const StepArgs& a, StepVariant v, hipStream_t st) {
    if (v.inplace == STREAM_NEIGHBOUR)
        return step_per<S, MON, FORM, false, CURVED, STREAM_NEIGHBOUR>(a, v.periodic_yz, st);
    return step_per<S, MON, FORM, false, CURVED, STREAM_LOCAL>(a, v.periodic_yz, st);
}

template <class S, bool MON, bool CURVED>
hipError_t step_form_inplace(const StepArgs& a, StepVariant v, hipStream_t st) {
    if (v.srt2) return step_inplace<S, MON, 2, CURVED>(a, v, st);
    return v.rates_one ? step_inplace<S, MON, 1, CURVED>(a, v, st) : step_inplace<S, MON, 0, CURVED>(a, v, st);
}

template <class S, bool CURVED>
hipError_t step_mon_inplace(const StepArgs& a, StepVariant v, hipStream_t st) {
    return v.monitor ? step_form_inplace<S, true, CURVED>(a, v, st) : step_form_inplace<S, false, CURVED>(a, v, st);
}

template <class S, bool MON, bool NT, bool CURVED>
hipError_t step_form(const StepArgs& a, StepVariant v, hipStream_t st) {
    if (v.srt2) return step_per<S, MON, 2, NT, CURVED>(a, v.periodic_yz, st);
    return v.rates_one ? step_per<S, MON, 1, NT, CURVED>(a, v.periodic_yz, st)
                       : step_per<S, MON, 0, NT, CURVED>(a, v.periodic_yz, st);
}

template <class S, bool NT, bool CURVED>
hipError_t step_mon(const StepArgs& a, StepVariant v, hipStream_t st) {
    return v.monitor ? step_form<S, true, NT, CURVED>(a, v, st) : step_form<S, false, NT, CURVED>(a, v, st);
}

template <class S, bool NT>
hipError_t step_nt(const StepArgs& a, StepVariant v, hipStream_t st) {
    return v.curved ? step_mon<S, NT, true>(a, v, st) : step_mon<S, NT, false>(a, v, st);
}

// Streaming stores only pay for 4- and 8-byte populations (measured); the
// 2-byte forms always store normally.
template <class S>
hipError_t step_t(const StepArgs& a, StepVariant v, hipStream_t st) {
    if (v.inplace != STREAM_PULL) {
        if (v.curved && a.cside == nullptr) return hipErrorInvalidValue;
        return v.curved ? step_mon_inplace<S, true>(a, v, st) : step_mon_inplace<S, false>(a, v, st);
    }
    if constexpr (sizeof(S) >= 4) {
        if (v.stream_store) return step_nt<S, true>(a, v, st);
    }
    return step_nt<S, false>(a, v, st);
}

}  // namespace

#if !defined(LBM_STEP_STORAGE)
#error "compile with -DLBM_STEP_STORAGE=0..3"
#elif LBM_STEP_STORAGE == 0
#define LBM_STEP_T double
#elif LBM_STEP_STORAGE == 1
#define LBM_STEP_T float
#elif LBM_STEP_STORAGE == 2
#define LBM_STEP_T _Float16
#else
#define LBM_STEP_T __bf16
#endif

hipError_t launch_step_s(const StepArgs& a, StepVariant v, hipStream_t stream,
                         std::integral_constant<int, LBM_STEP_STORAGE>) {
    return step_t<LBM_STEP_T>(a, v, stream);
}

hipError_t launch_inplace_reverse_s(const StepArgs& a, bool fill_side, hipStream_t stream,
                                    std::integral_constant<int, LBM_STEP_STORAGE>) {
    if (a.n <= 0) return hipSuccess;
    if (fill_side && (a.cside == nullptr || a.crec == nullptr)) return hipErrorInvalidValue;
    const dim3 grid((a.n + BLOCK - 1) / BLOCK), block(BLOCK);
    if (!fill_side) hipLaunchKernelGGL((k_inplace_reverse<LBM_STEP_T, false, false>), grid, block, 0, stream, a);
    else if (a.periodic & 6) hipLaunchKernelGGL((k_inplace_reverse<LBM_STEP_T, true, true>), grid, block, 0, stream, a);
    else hipLaunchKernelGGL((k_inplace_reverse<LBM_STEP_T, false, true>), grid, block, 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_inplace_unstream_s(const StepArgs& a, hipStream_t stream, std::integral_constant<int, LBM_STEP_STORAGE>) {
    if (a.n <= 0) return hipSuccess;
    const dim3 grid((a.n + BLOCK - 1) / BLOCK), block(BLOCK);
    if (a.periodic & 6) hipLaunchKernelGGL((k_inplace_unstream<LBM_STEP_T, true>), grid, block, 0, stream, a);
    else hipLaunchKernelGGL((k_inplace_unstream<LBM_STEP_T, false>), grid, block, 0, stream, a);
    return hipGetLastError();
}

}  // namespace lbm
