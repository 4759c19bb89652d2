// Host-side internals of the library shared by the domain API (lbm_api.cpp)
// and the batch API (lbm_batch_api.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

namespace lbm_host {

// Error reporting: the message is kept per thread for lbm_last_error().
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
bool finite_all(const double* v, int n);

constexpr int GRAPH_STEPS = 16;   // even, so a replay returns to the same buffer parity
// Population working sets above this size do not stay in the 256 MB Infinity
// Cache; there streaming (non-temporal) stores are faster.
constexpr size_t STREAM_STORE_BYTES = (size_t)192 << 20;
// LBM_STREAM_AUTO streams 4- and 8-byte populations in place where the two
// buffers of the pull scheme exceed STREAM_STORE_BYTES and one buffer is at
// most this size (measured at the aneurysm: in place gains 15-23 % for FP32
// at 105-218 MiB per buffer, 16 % and 7 % for FP64 at 209 and 293 MiB, and
// loses 11 % for FP64 at 437 MiB; the 2-byte forms lose 10 % at 52-109 MiB).
constexpr size_t INPLACE_MAX_BYTES = (size_t)320 << 20;

}  // namespace lbm_host

#define HIP_TRY(expr, what)                                            \
    do {                                                               \
        hipError_t _e = (expr);                                        \
        if (_e != hipSuccess) return lbm_host::hip_fail(_e, what);     \
    } while (0)

// Layout of an in-place domain's population buffer (lbm::STREAM_PULL has the
// description of the reversed and streamed layouts).
enum : int { LAYOUT_PULL = 0, LAYOUT_REVERSED = 1, LAYOUT_STREAMED = 2 };

// A domain: host tables, parameters, the layout of its device memory and its
// time/buffer bookkeeping.
struct lbm_domain {
    int nx = 0, ny = 0, nz = 0;
    unsigned periodic = 0;
    int storage = 0;
    hipStream_t stream = nullptr;

    int64_t n = 0;
    int npad = 0;
    int W = 0;
    int rows = 0;
    int nblocks = 0, blocks_per_xcd = 0;
    int row_tile = 0;                      // row-tile edge of the node order
    std::vector<uint32_t> node_words;      // [npad]
    std::vector<uint32_t> wave_special;    // [npad / 64] chunks holding a special node
    std::vector<lbm::RowEntry> rowtab;     // [rows][W]
    std::vector<lbm::SpecialNode> spec;
    std::vector<int32_t> spec_plane;       // [nspec][27] plane of each pulled value
    std::vector<int32_t> link_meta;        // [nlinks] type | alpha << 8
    std::vector<double> link_coef;         // [nlinks][LINK_COEFS]
    std::vector<int32_t> link_xyz;         // [nlinks][3] node coordinates of each link
    // curved-wall weights (signed w0, layout at lbm::CREC_CHUNK; empty for
    // halfway walls) and the first record of each 64-node chunk
    std::vector<double> crec;
    std::vector<float> crec_f32;           // the same in FP32 (storage other than f64)
    std::vector<uint32_t> crec_base;
    std::vector<int32_t> coords;           // [n][3]
    bool has_inlet_links = false;
    size_t nlinks() const { return link_meta.size(); }

    // parameters
    bool params_set = false;
    double tau = 0.0, s[4] = {1, 1, 1, 1}, g[3] = {0, 0, 0};
    double rho_out = 1.0;
    bool inlet_set = false;
    double axis[3] = {0, 0, 1}, center[3] = {0, 0, 0}, radius = 0, G0 = 0, G1 = 0, omega = 0;
    bool links_dirty = true;

    // device memory
    char* dev = nullptr;
    size_t dev_bytes = 0;
    size_t off_popA = 0, off_popB = 0, off_node = 0, off_rowtab = 0, off_spec = 0, off_lmeta = 0,
           off_lcoef = 0, off_ladd = 0, off_tcount = 0, off_trig = 0, off_part = 0, off_monout = 0, off_avg = 0,
           off_probe = 0, off_crec = 0, off_cbase = 0, off_cside = 0, off_wspec = 0;
    size_t pop_bytes = 0;

    // cur: time-counter slot of the next step, toggled by every step.  The
    // population buffer read next is A when cur ^ pop_flip == 0, else B: a
    // pull step moves to the other buffer with cur; an in-place step stays by
    // toggling pop_flip with it.
    int cur = 0;
    int pop_flip = 0;
    int stream_mode = LBM_STREAM_AUTO;   // lbm_set_streaming
    int layout = 0;           // the buffer's layout: LAYOUT_PULL, LAYOUT_REVERSED or LAYOUT_STREAMED
    int64_t t = 0;
    int64_t t_upload[2] = {0, 0};
    double trig_host[4] = {1, 0, 1, 0};   // (cos, sin)(omega t) for slots t & 1
    bool initialized = false;
    bool monitored = false;   // a monitored step ran since initialisation
    int mon_blocks = 0;       // monitor partials written by that step
    int64_t avg_count = 0;
    bool avg_track = false;   // the step kernel adds u of every step to the accumulator
    // monitoring points
    int nprobe = 0, probe_every = 1;
    double* probe_out = nullptr;
    int64_t probe_t0 = 0, probe_cap = 0;
    double mon_host[lbm::MON_WORDS] = {0};

    // Captured graphs of GRAPH_STEPS consecutive steps, one per starting state
    // (graph_key: time slot, buffer choice, layout).  Kernel arguments are baked
    // in, so any parameter change drops them.
    static constexpr int NGRAPH = 12;
    hipGraphExec_t graph[NGRAPH] = {};
    int graph_key() const { return cur | (pop_flip << 1) | (layout << 2); }

    void drop_graphs() {
        for (auto& g : graph) {
            if (g) hipGraphExecDestroy(g);
            g = nullptr;
        }
    }
    ~lbm_domain() { drop_graphs(); }

    int64_t cell(int x, int y, int z) const { return ((int64_t)z * ny + y) * nx + x; }
    int row_of(int y, int z) const { return (z + 1) * (ny + 2) + (y + 1); }
    // index of the fluid node at (x, y, z) (must be fluid): prefix + popcount
    // of the entry's cells 30k - 1 .. x - 1
    bool is_fluid(int x, int y, int z) const {
        const int k = x / lbm::ROW_SPAN, r = x - k * lbm::ROW_SPAN;
        return (rowtab[(size_t)row_of(y, z) * W + k].bits >> (r + 1)) & 1u;
    }
    int32_t index_of(int x, int y, int z) const {
        const int k = x / lbm::ROW_SPAN, r = x - k * lbm::ROW_SPAN;
        const lbm::RowEntry& e = rowtab[(size_t)row_of(y, z) * W + k];
        return e.prefix + __builtin_popcount(e.bits & ((2u << r) - 1u));
    }
    int collision = 0;                     // LBM_COLLISION_*
    // the CHM-MRT form with every free rate equal to one (its specialized kernel)
    bool rates_one() const {
        return collision == 0 && s[0] == 1.0 && s[1] == 1.0 && s[2] == 1.0 && s[3] == 1.0;
    }
    bool periodic_yz() const { return (periodic & 6u) != 0; }
    // whether lbm_step streams in place (LBM_STREAM_AUTO: see lbm.h)
    bool use_inplace() const;
};

namespace lbm_host {

// Kernel arguments for the domain's current buffer parity.
lbm::StepArgs make_args(const lbm_domain* d);
// Upload the open-boundary coefficients and inlet phase if they changed.
int prepare_links(lbm_domain* d);
// Bring an in-place domain's populations back to the pull layout (the layout
// every reader of the state and the pull batch use); a no-op for the pull layout.
int sync_pull(lbm_domain* d);
// Pull layout -> reversed layout, in place (the first in-place step reads it).
int enter_inplace(lbm_domain* d);

}  // namespace lbm_host
