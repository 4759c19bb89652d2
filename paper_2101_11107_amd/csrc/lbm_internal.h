// Internal declarations shared by the host side (lbm_api.cpp) and the HIP
// kernels (lbm_kernels.hip) of the library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace lbm {

// Fluid-node descriptor word.  Ordinary node: x | y << 10 | z << 20.
// Node that needs the general path (an open-boundary link or a link that wraps
// around a periodic x axis): SPECIAL_BIT | index into the special table.
constexpr uint32_t SPECIAL_BIT = 0x80000000u;
constexpr int MAX_DIM = 1023;
constexpr int BLOCK = 256;            // threads per work-group of the step kernel
constexpr int MON_WORDS = 10;         // doubles per work-group monitor partial

// Source code of one incoming link of a special node.
//   >= 0  : index of the fluid node the population is pulled from
//   -1    : wall (halfway bounce-back)
//   <= -2 : open-boundary link, index (-2 - code) into the link table
constexpr int32_t SRC_WALL = -1;

struct alignas(16) SpecialNode {
    int32_t node;          // fluid-node index
    int32_t x, y, z;
    int32_t src[27];
    int32_t pad;
};
static_assert(sizeof(SpecialNode) == 128, "special node record is 128 bytes");

enum : int32_t { LINK_INLET = 2, LINK_OUTLET = 3 };

struct alignas(16) BcLink {
    int32_t type;          // LINK_INLET or LINK_OUTLET
    int32_t pad;
    double a0;             // inlet: steady axial speed at the link midpoint
    double a1re, a1im;     // inlet: complex oscillating amplitude
};
static_assert(sizeof(BcLink) == 32, "link record is 32 bytes");

// Kernel arguments of one step over one domain (passed by value).
struct StepArgs {
    const void* fin;             // post-collision populations of time t  [27][npad]
    void* fout;                  // post-collision populations of time t+1
    const uint32_t* node;        // [npad] descriptor words
    const uint32_t* bits;        // [rows][W] fluid bitmap, bit (x + 1) of row (y, z)
    const int32_t* prefix;       // [rows][W] fluid nodes before each bitmap word
    const SpecialNode* spec;     // [nspec]
    const BcLink* links;         // [nlinks]
    double* u_spec;              // [nspec][3] velocity of each special node's last collision
    int64_t* tcount;             // [2] time counters (read slot tin, write slot tin ^ 1)
    double* partials;            // [nblocks][MON_WORDS] monitor partials
    int tin;
    int n, npad, nx, ny, nz, W, periodic;
    int nblocks, blocks_per_xcd;
    double s[5];                 // relaxation rates of orders 2..6
    double g[3];                 // body acceleration
    double omega;                // inlet angular frequency
    double axis[3];              // inlet direction (unit)
    double rho_out;              // outlet density
};

// Launchers (lbm_kernels.hip).  All enqueue on `stream` and return the HIP status.
hipError_t launch_step(int storage, const StepArgs& a, bool full, hipStream_t stream);
hipError_t launch_init(int storage, const StepArgs& a, const double* rho, const double* u,
                       hipStream_t stream);
hipError_t launch_moments(int storage, const StepArgs& a, double* rho, double* u, double* avg,
                          int avg_mode, double avg_count, hipStream_t stream);
hipError_t launch_read_populations(int storage, const StepArgs& a, double* out, hipStream_t stream);
hipError_t launch_monitor_finalize(const double* partials, int nblocks, double* out,
                                   hipStream_t stream);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t stream);

}  // namespace lbm
