// Internal declarations shared by the host side (lbm_api.cpp,
// lbm_batch_api.cpp) and the HIP kernels (lbm_step.hip, lbm_batch.hip,
// lbm_kernels.hip) of the library.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <type_traits>

namespace lbm {

// Fluid-node descriptor word (32 bits).
//  - ordinary node, no periodic y/z axis: x | row << 10, row = (z+1)(ny+2) + (y+1)
//  - ordinary node, periodic y or z axis:  x | y << 10 | z << 20
//  - node that needs the general path (an open-boundary link, or a link that
//    wraps around a periodic x axis): SPECIAL_BIT | index into the special table
constexpr uint32_t SPECIAL_BIT = 0x80000000u;
constexpr int MAX_DIM = 1023;
constexpr int BLOCK = 256;            // threads per work-group of the step kernel
constexpr int MON_WORDS = 10;         // doubles per work-group monitor partial

// Population layout: tiles of 256-byte runs.  T = 256 / size consecutive
// nodes (128 for 2-byte storage, 64 in FP32, 32 in FP64) form a tile that
// holds their 27 directions one after another, each as one run of T
// consecutive values, so element (node i, direction a) is at
// (i / T) 27 T + a T + i % T.  A wave's loads and stores of one direction
// then cover whole runs, and the 27 runs of a tile are adjacent in memory.
// (With 64-node runs of 2-byte values, single 128-byte lines, one plane per
// direction measured faster; 256-byte runs measured 3 % faster than planes.)
// npad is a multiple of 256, so every tile is whole.
constexpr uint32_t POP_RUN_BYTES = 256;
__host__ __device__ __forceinline__ constexpr uint32_t pop_tile_shift(uint32_t sz) {
    return sz == 8 ? 5u : (sz == 4 ? 6u : 7u);
}
__host__ __device__ __forceinline__ constexpr uint32_t pop_index(uint32_t i, uint32_t a, uint32_t npad, uint32_t sz) {
    (void)npad;
    return (i >> pop_tile_shift(sz)) * (27u << pop_tile_shift(sz)) + (a << pop_tile_shift(sz)) +
           (i & ((1u << pop_tile_shift(sz)) - 1u));
}

// Row table entry k of a row: fluid bits of the 32 cells 30k - 1 .. 30k + 30
// (bit j for cell 30k - 1 + j; neighbouring entries overlap by two cells, so
// the cells x - 1, x, x + 1 of any x in 30k .. 30k + 29 sit in entry k) and the
// list index of the row's first fluid cell at or after 30k - 1 (the number
// of fluid nodes before it in list order).
constexpr int ROW_SPAN = 30;          // cells per row-table entry
constexpr int MAX_PROBES = 64;        // monitoring points of a domain
struct alignas(8) RowEntry {
    uint32_t bits;
    int32_t prefix;
};

// Record of a node with open-boundary or periodic-x links.  off[alpha] is the
// byte offset (from the population buffer) of the value it pulls: the source
// node's alpha population for a fluid link, its own abar population for a wall
// or open link (bounce-back).  Open links then get the boundary correction:
// inlet f += add, outlet f = -f + add.  The node's open links are numbered
// from link0 in increasing alpha.  Its wall links (wallmask) are blended after
// the gather like those of ordinary nodes when the domain has curved walls.
struct alignas(16) SpecialNode {
    uint32_t off[27];
    int32_t node;          // fluid-node index
    int32_t link0;         // first link of this node
    uint32_t wallmask;     // bit alpha: wall link
    uint32_t linkmask;     // bit alpha: open-boundary link
    uint32_t reserved;
};
static_assert(sizeof(SpecialNode) == 128, "special node record is 128 bytes");

enum : int32_t { LINK_INLET = 2, LINK_OUTLET = 3 };

// Curved-wall weights (Eq. (9)-(10)), blended into the step after the
// gather.  One weight r per wall link of a node, stored in the population's
// arithmetic type: grouped by chunk of 64
// consecutive nodes (one wavefront), inside a chunk by incoming direction
// alpha, inside a direction by node; crec_base[chunk] is the chunk's first
// record.  |r| = w0 is the weight of the bounce-back value f*_abar(x) and
// 1 - w0 that of the second value: for r > 0 (q < 1/2) f*_abar(x + c_alpha),
// which the node pulls for direction abar anyway; for r < 0 (q >= 1/2) the
// node's own f*_alpha(x).  Wall links without a distance have r = 1 (halfway
// bounce-back).
constexpr int CREC_CHUNK = 64;

// Per open-boundary link: meta = type | alpha << 8; coef = (a0, a1re, a1im,
// k1, k3, k5): the inlet speed at the link midpoint is
// U = a0 + a1re cos(omega t) - a1im sin(omega t), and the moving-wall term
// f_eq_a(1, axis U) - f_eq_abar(1, axis U) equals the odd polynomial
// U (k1 + U^2 (k3 + U^2 k5)) exactly; add = additive term of the incoming
// population for the next step (inlet: that moving-wall term; outlet:
// f_eq_a + f_eq_abar - 2 w_a at rho_out and the node's velocity).
constexpr int LINK_COEFS = 6;
struct StepArgs {
    const void* fin;             // post-collision populations of time t (pop_index layout, npad nodes)
    void* fout;                  // post-collision populations of time t+1
    const uint32_t* node;        // [npad] descriptor words
    const uint32_t* wave_special; // [npad / 64] non-zero where the 64-node chunk holds a special node
    const RowEntry* rowtab;      // [rows][W]
    const SpecialNode* spec;     // [nspec]
    const int32_t* link_meta;    // [nlinks]
    const double* link_coef;     // [nlinks][LINK_COEFS]
    double* link_add;            // [nlinks]
    const void* crec;            // curved-wall weights, or null (halfway walls)
    const uint32_t* crec_base;   // [npad / CREC_CHUNK] first record of each 64-node chunk
    void* cside;                 // curved walls streamed in place: per record, the node's own
                                 // post-collision f*_alpha of the last step (storage type)
    int64_t* tcount;             // [2] time counters (read slot tin, write slot tin ^ 1)
    double* trig;                // [2][2] (cos, sin)(omega t), slot t & 1
    double* partials;            // [nblocks][MON_WORDS] monitor partials
    double* avg;                 // [3][n] FP64 velocity sums the step adds to, or null
    const int32_t* probe_node;   // [nprobe] node indices of the monitoring points
    double* probe_out;           // [probe_cap][nprobe][4] (rho, ux, uy, uz) records, or null
    int64_t probe_t0, probe_cap; // time the probes were set; records the buffer holds
    int nprobe, probe_every;     // probes (0: none); record every probe_every steps
    int tin;
    int collision;               // LBM_COLLISION_CHM_MRT or LBM_COLLISION_SRT2
    int n, npad, nx, ny, nz, W, periodic;
    int nblocks, blocks_per_xcd;
    double s[5];                 // relaxation rates of orders 2..6
    double g[3];                 // body acceleration
    double omega;                // inlet angular frequency
    double cos_w, sin_w;         // cos(omega), sin(omega): one-step rotation of the inlet phase
    double axis[3];              // inlet direction (unit)
    double rho_out;              // outlet density
};

// Kernel variant of a step: which collision and which monitors.
struct StepVariant {
    bool monitor;        // accumulate the FP64 monitors (mass, momentum, wall force, fluxes)
    bool rates_one;      // free rates of orders 3..6 all equal to 1
    bool periodic_yz;    // a periodic y or z axis (node words hold x, y, z)
    bool stream_store;   // non-temporal population stores (working set beyond the Infinity Cache)
    bool srt2;           // the SRT comparator instead of CHM-MRT
    bool curved;         // curved-wall weights (crec set)
    int inplace;         // 0: pull between two buffers; in-place streaming (fin == fout): 1 the
                         // neighbour step, 2 the node-local step (STREAM_* below)
};

// In-place (AA-pattern) streaming keeps one population buffer.  Its layouts:
//  * reversed (R): the post-collision f*_a(x) of the last step in slot abar of
//    node x, i.e. the pull layout with every node's slots reversed;
//  * streamed (S): slot a of node x holds the value that arrives there,
//    f*_a(x - c_a) from a fluid neighbour, or the node's own f*_abar(x) where
//    x - c_a is not fluid (bounce-back and open links, before their rules).
// The neighbour step reads R (direction a of x at (x - c_a, abar), or at
// (x, a) on a wall or open link) and writes f*_abar of x to that same place,
// leaving S; the node-local step reads slot a of x and writes f*_a to slot
// abar, leaving R.  Each location is read and written by one thread only.
enum : int { STREAM_PULL = 0, STREAM_NEIGHBOUR = 1, STREAM_LOCAL = 2 };

// Several domains stepped by one launch.  Work item k of the launch is block
// (item_map[k] & ITEM_BLOCK_MASK) of domain (item_map[k] >> ITEM_DOMAIN_SHIFT);
// doms[d] holds the domain's arguments for its buffer parity at the start of
// the launch sequence (odd steps swap the buffers and the time slot).
constexpr int MAX_PERSISTENT_GROUPS = 4096;              // work-groups of one persistent launch
constexpr int BARRIER_WORDS = 64 + MAX_PERSISTENT_GROUPS;   // release word, padding, arrivals
constexpr int ITEM_DOMAIN_SHIFT = 20;
constexpr int ITEM_BLOCK_MASK = (1 << ITEM_DOMAIN_SHIFT) - 1;
struct BatchArgs {
    const StepArgs* doms;        // [ndom]
    const int* item_map;         // [nitems]
    int ndom, nitems, items_per_xcd;
    unsigned* barrier;           // [BARRIER_WORDS] device-wide barrier words (persistent mode)
    int* error;                  // set when a device-wide barrier wait exceeded its bound
};

// Execution choices of a batch (picked by the autotuner).
struct BatchConfig {
    int mode;            // 0: one launch per step; 1: persistent launch with device-wide barriers;
                         // 2: one launch per step, streamed in place (BATCH_MODE_INPLACE)
    int block;           // work-group size: 128, 256 or 512
    int stream_store;    // non-temporal population stores
    int grid;            // persistent mode: number of work-groups (0 = all that fit)
    int group_mb;        // domains stepped together per group, by population working set (0 = all)
};

// Launchers (lbm_kernels.hip; launch_step dispatches to the per-storage step
// launchers of lbm_step.hip).  All enqueue on `stream` and return the HIP status.
hipError_t launch_step(int storage, const StepArgs& a, StepVariant v, hipStream_t stream);
// The step launcher of one storage type (lbm_step.hip, one translation unit each).
hipError_t launch_step_s(const StepArgs& a, StepVariant v, hipStream_t stream, std::integral_constant<int, 0>);
hipError_t launch_step_s(const StepArgs& a, StepVariant v, hipStream_t stream, std::integral_constant<int, 1>);
hipError_t launch_step_s(const StepArgs& a, StepVariant v, hipStream_t stream, std::integral_constant<int, 2>);
hipError_t launch_step_s(const StepArgs& a, StepVariant v, hipStream_t stream, std::integral_constant<int, 3>);
hipError_t launch_inplace_reverse_s(const StepArgs& a, bool fill_side, hipStream_t stream, std::integral_constant<int, 0>);
hipError_t launch_inplace_reverse_s(const StepArgs& a, bool fill_side, hipStream_t stream, std::integral_constant<int, 1>);
hipError_t launch_inplace_reverse_s(const StepArgs& a, bool fill_side, hipStream_t stream, std::integral_constant<int, 2>);
hipError_t launch_inplace_reverse_s(const StepArgs& a, bool fill_side, hipStream_t stream, std::integral_constant<int, 3>);
hipError_t launch_inplace_unstream_s(const StepArgs& a, hipStream_t stream, std::integral_constant<int, 0>);
hipError_t launch_inplace_unstream_s(const StepArgs& a, hipStream_t stream, std::integral_constant<int, 1>);
hipError_t launch_inplace_unstream_s(const StepArgs& a, hipStream_t stream, std::integral_constant<int, 2>);
hipError_t launch_inplace_unstream_s(const StepArgs& a, hipStream_t stream, std::integral_constant<int, 3>);
hipError_t launch_init(int storage, const StepArgs& a, const double* rho, const double* u,
                       hipStream_t stream);
hipError_t launch_moments(int storage, const StepArgs& a, double* rho, double* u, double* avg,
                          int avg_mode, double avg_count, hipStream_t stream);
hipError_t launch_read_populations(int storage, const StepArgs& a, double* out, hipStream_t stream);
// In-place streaming layouts to and from the pull layout (lbm_step.hip):
// reverse swaps every node's slots a and abar of a.fin in place (pull <-> R;
// fill_side, from the pull layout: also copy each curved-wall link's own
// f*_alpha into a.cside); unstream writes the pull layout of the S state in
// a.fin into a.fout.
hipError_t launch_inplace_reverse(int storage, const StepArgs& a, bool fill_side, hipStream_t stream);
hipError_t launch_inplace_unstream(int storage, const StepArgs& a, hipStream_t stream);
hipError_t launch_monitor_finalize(const double* partials, int nblocks, double* out,
                                   hipStream_t stream);
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t stream);

// Batched launchers (lbm_batch.hip).  kind: BATCH_RATES_ONE when every domain
// is CHM-MRT with free rates of one, | BATCH_CURVED when a domain has
// curved-wall records, | BATCH_IP_NEIGHBOUR or BATCH_IP_LOCAL for the
// in-place kind of this launch (BATCH_MODE_INPLACE only, which takes 256
// threads, cached stores and no curved walls); step: the step index within the
// launch sequence (its parity selects the time slot and, for pull, the
// buffers); monitor: accumulate monitors.
enum : int { BATCH_RATES_ONE = 1, BATCH_CURVED = 2, BATCH_IP_NEIGHBOUR = 4, BATCH_IP_LOCAL = 8 };
enum : int { BATCH_MODE_STEP = 0, BATCH_MODE_PERSISTENT = 1, BATCH_MODE_INPLACE = 2 };
hipError_t launch_batch_step(int storage, int kind, const BatchArgs& b, const BatchConfig& c, int step,
                             bool monitor, hipStream_t stream);
hipError_t launch_batch_persistent(int storage, int kind, const BatchArgs& b, const BatchConfig& c,
                                   int step0, int nsteps, hipStream_t stream);
// Work-groups of the persistent kernel that fit on the device at once.
hipError_t batch_persistent_capacity(int storage, int kind, const BatchConfig& c, int* blocks);
// One definition per storage type, each in its own translation unit; the
// functions above dispatch to them.
#define LBM_BATCH_DECL(K)                                                                                  \
    hipError_t launch_batch_step_s(int storage, int kind, const BatchArgs& b, const BatchConfig& c,   \
                                   int step, bool monitor, hipStream_t stream, std::integral_constant<int, K>); \
    hipError_t launch_batch_persistent_s(int storage, int kind, const BatchArgs& b,                  \
                                         const BatchConfig& c, int step0, int nsteps, hipStream_t stream,   \
                                         std::integral_constant<int, K>);                                   \
    hipError_t batch_persistent_capacity_s(int storage, int kind, const BatchConfig& c, int* blocks,  \
                                           std::integral_constant<int, K>);
LBM_BATCH_DECL(0)
LBM_BATCH_DECL(1)
LBM_BATCH_DECL(2)
LBM_BATCH_DECL(3)
#undef LBM_BATCH_DECL

}  // namespace lbm
