// C ABI of batched stepping: many domains advanced together by launches that
// cover all of them, captured into graphs, with an autotuner that times the
// execution choices (one launch per step or a persistent launch, work-group
// size, streaming stores, persistent grid size) on the batch itself.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "lbm.h"
#include "lbm_host.h"
#include "lbm_internal.h"

using namespace lbm_host;

struct lbm_batch {
    std::vector<lbm_domain*> doms;
    hipStream_t stream = nullptr;
    int storage = 0;
    bool rates_one = true;
    int64_t total_nodes = 0;

    char* dev = nullptr;
    size_t dev_bytes = 0;
    size_t off_args = 0, off_items = 0, off_barrier = 0, off_error = 0;

    // Groups of consecutive domains stepped together (cache blocking): group g
    // covers domains [group_first[g], group_first[g+1]); its work-item table
    // starts at items_host[item_off[g]].
    std::vector<int> group_first;
    std::vector<int> item_off;
    std::vector<int> group_items;

    std::vector<lbm::StepArgs> args_host;
    std::vector<int> items_host;
    std::vector<int> built_parity;    // each domain's buffer parity when args_host was built
    int built_block = 0, built_group_mb = -1, built_mode = -1;
    int built_layout = -1;             // the domains' layout when args_host was built

    lbm::BatchConfig cfg{0, 256, 0, 0, 0};
    std::vector<hipGraphExec_t> graphs;   // per group: GRAPH_STEPS steps with cfg
    int graph_cfg[7] = {-1, -1, -1, -1, -1, -1, -1};
    int error_host = 0;

    void drop_graph() {
        for (auto& g : graphs)
            if (g) hipGraphExecDestroy(g);
        graphs.clear();
    }
    ~lbm_batch() { drop_graph(); }
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

lbm::BatchArgs batch_args(const lbm_batch* b, int g) {
    lbm::BatchArgs a{};
    a.doms = (const lbm::StepArgs*)(b->dev + b->off_args) + b->group_first[g];
    a.item_map = (const int*)(b->dev + b->off_items) + b->item_off[g];
    a.ndom = b->group_first[g + 1] - b->group_first[g];
    a.nitems = b->group_items[g];
    a.items_per_xcd = (a.nitems + 7) / 8;
    a.barrier = (unsigned*)(b->dev + b->off_barrier);
    a.error = (int*)(b->dev + b->off_error);
    return a;
}

// Bring every domain to the layout the configuration steps: the pull layout,
// or one in-place layout shared by all domains (kept when they already share
// one, else every domain enters the reversed layout from the pull layout).
// The conversions run on the domains' streams, after the batch's own earlier
// work has finished.
int align_layouts(lbm_batch* b) {
    const bool inplace = b->cfg.mode == lbm::BATCH_MODE_INPLACE;
    const int l0 = b->doms[0]->layout;
    bool same = inplace ? l0 != LAYOUT_PULL : l0 == LAYOUT_PULL;
    for (const lbm_domain* d : b->doms) same = same && d->layout == l0;
    if (same) return LBM_OK;
    HIP_TRY(hipStreamSynchronize(b->stream), "batch stream synchronize");
    for (lbm_domain* d : b->doms) {
        int rc = sync_pull(d);
        if (rc == LBM_OK && inplace) rc = enter_inplace(d);
        if (rc) return rc;
    }
    return LBM_OK;
}

// Bring the device tables up to date with the domains' parities and layouts
// and the block size of the current configuration.
int refresh_tables(lbm_batch* b) {
    int rc = align_layouts(b);
    if (rc) return rc;
    bool stale = b->built_block != b->cfg.block || b->built_parity.size() != b->doms.size() ||
                 b->built_mode != b->cfg.mode || b->built_layout != b->doms[0]->layout;
    for (size_t k = 0; !stale && k < b->doms.size(); ++k) stale = b->built_parity[k] != b->doms[k]->cur;
    for (lbm_domain* d : b->doms) {
        if (d->links_dirty) stale = true;
        rc = prepare_links(d);
        if (rc) return rc;
        // the domain's own stream may hold its uploads; the batch runs on its own stream
        HIP_TRY(hipStreamSynchronize(d->stream), "domain stream synchronize");
    }
    if (b->built_group_mb != b->cfg.group_mb) stale = true;
    // any change of a domain's kernel arguments (parameters, boundary data,
    // velocity tracking) since the tables were built
    for (size_t k = 0; !stale && k < b->doms.size(); ++k) {
        const lbm::StepArgs now = make_args(b->doms[k]);
        stale = std::memcmp(&now, &b->args_host[k], sizeof now) != 0;
    }
    if (!stale) return LBM_OK;
    const int bs = b->cfg.block;
    // Groups of consecutive domains: as many as the working-set budget asks
    // for (the population buffers each domain steps: two with pull, one in
    // place), with boundaries at the domain edges closest to equal shares, so
    // no group is left small (a small launch runs below the bandwidth of a
    // large one).
    const size_t nd = b->doms.size();
    const double buffers = b->cfg.mode == lbm::BATCH_MODE_INPLACE ? 1.0 : 2.0;
    std::vector<double> cum(nd + 1, 0.0);
    for (size_t k = 0; k < nd; ++k) cum[k + 1] = cum[k] + buffers * (double)b->doms[k]->pop_bytes;
    const double budget = b->cfg.group_mb > 0 ? (double)((size_t)b->cfg.group_mb << 20) : 0.0;
    const size_t ngroups = budget > 0.0 ? std::min(nd, (size_t)std::ceil(cum[nd] / budget)) : 1;
    b->group_first.assign(1, 0);
    for (size_t g = 1; g < ngroups; ++g) {
        const double target = cum[nd] * (double)g / (double)ngroups;
        size_t k = (size_t)b->group_first.back() + 1;
        while (k < nd && cum[k] < target) ++k;
        if (k > (size_t)b->group_first.back() + 1 && target - cum[k - 1] < cum[k] - target) --k;
        // keep at least one domain for each group still to come
        k = std::min(k, nd - (ngroups - g));
        b->group_first.push_back((int)k);
    }
    b->group_first.push_back((int)nd);
    const int ng = (int)b->group_first.size() - 1;
    b->args_host.resize(b->doms.size());
    b->built_parity.resize(b->doms.size());
    b->items_host.clear();
    b->item_off.assign(ng, 0);
    b->group_items.assign(ng, 0);
    for (int g = 0; g < ng; ++g) {
        b->item_off[g] = (int)b->items_host.size();
        for (int k = b->group_first[g]; k < b->group_first[g + 1]; ++k) {
            lbm_domain* d = b->doms[k];
            b->args_host[k] = make_args(d);
            b->built_parity[k] = d->cur;
            const int blocks = (int)((d->n + bs - 1) / bs);
            const int local = k - b->group_first[g];
            for (int q = 0; q < blocks; ++q) b->items_host.push_back((local << lbm::ITEM_DOMAIN_SHIFT) | q);
        }
        b->group_items[g] = (int)b->items_host.size() - b->item_off[g];
    }
    b->built_block = bs;
    b->built_group_mb = b->cfg.group_mb;
    b->built_mode = b->cfg.mode;
    b->built_layout = b->doms[0]->layout;
    b->drop_graph();
    HIP_TRY(hipMemcpyAsync(b->dev + b->off_args, b->args_host.data(), b->args_host.size() * sizeof(lbm::StepArgs),
                           hipMemcpyHostToDevice, b->stream), "batch table upload");
    HIP_TRY(hipMemcpyAsync(b->dev + b->off_items, b->items_host.data(), b->items_host.size() * sizeof(int),
                           hipMemcpyHostToDevice, b->stream), "batch table upload");
    return LBM_OK;
}

// Kernel flags of the batch: every domain CHM-MRT with free rates of one; some
// domain with curved-wall records.
int batch_kind(const lbm_batch* b) {
    int kind = b->rates_one ? lbm::BATCH_RATES_ONE : 0;
    for (const lbm_domain* d : b->doms)
        if (!d->crec.empty()) kind |= lbm::BATCH_CURVED;
    return kind;
}

// Enqueue nsteps (>= 1) steps of group g with the current configuration; the
// last one accumulates the group's monitors.  In place, the kinds alternate
// from the layout the tables were built at (reversed: the neighbour kind
// first).
int enqueue_steps(lbm_batch* b, int g, int nsteps) {
    const lbm::BatchArgs a = batch_args(b, g);
    if (b->cfg.mode == lbm::BATCH_MODE_INPLACE) {
        const bool rev0 = b->built_layout == LAYOUT_REVERSED;
        for (int s = 0; s < nsteps; ++s) {
            const int ip = (rev0 == ((s & 1) == 0)) ? lbm::BATCH_IP_NEIGHBOUR : lbm::BATCH_IP_LOCAL;
            HIP_TRY(lbm::launch_batch_step(b->storage, batch_kind(b) | ip, a, b->cfg, s, s == nsteps - 1, b->stream),
                    "batch step kernel");
        }
        return LBM_OK;
    }
    if (b->cfg.mode == lbm::BATCH_MODE_PERSISTENT && nsteps > 1) {
        // barrier epochs restart at 1 in every launch
        HIP_TRY(lbm::launch_fill_zero(a.barrier, lbm::BARRIER_WORDS * sizeof(unsigned), b->stream),
                "barrier reset");
        HIP_TRY(lbm::launch_batch_persistent(b->storage, batch_kind(b), a, b->cfg, 0, nsteps - 1, b->stream),
                "persistent batch kernel");
        HIP_TRY(lbm::launch_batch_step(b->storage, batch_kind(b), a, b->cfg, nsteps - 1, true, b->stream),
                "batch step kernel");
        return LBM_OK;
    }
    for (int s = 0; s < nsteps; ++s)
        HIP_TRY(lbm::launch_batch_step(b->storage, batch_kind(b), a, b->cfg, s, s == nsteps - 1, b->stream),
                "batch step kernel");
    return LBM_OK;
}

int ensure_graphs(lbm_batch* b) {
    const int key[7] = {b->cfg.mode, b->cfg.block, b->cfg.stream_store, b->cfg.grid, b->cfg.group_mb,
                        batch_kind(b), b->built_layout};
    const int ng = (int)b->group_first.size() - 1;
    if ((int)b->graphs.size() == ng && std::memcmp(key, b->graph_cfg, sizeof key) == 0) return LBM_OK;
    b->drop_graph();
    for (int g = 0; g < ng; ++g) {
        hipGraph_t gr = nullptr;
        HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed), "graph capture begin");
        int rc = enqueue_steps(b, g, GRAPH_STEPS);
        hipError_t e = hipStreamEndCapture(b->stream, &gr);
        if (rc) {
            if (gr) hipGraphDestroy(gr);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "graph capture end");
        hipGraphExec_t ex = nullptr;
        e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        hipGraphDestroy(gr);
        if (e != hipSuccess) return hip_fail(e, "graph instantiate");
        b->graphs.push_back(ex);
    }
    std::memcpy(b->graph_cfg, key, sizeof key);
    return LBM_OK;
}

void advance_domains(lbm_batch* b, int nsteps) {
    for (lbm_domain* d : b->doms) {
        d->cur ^= (nsteps & 1);
        // in place: one buffer, and the layout turns with every step
        if (d->layout != LAYOUT_PULL && (nsteps & 1)) {
            d->pop_flip ^= 1;
            d->layout = LAYOUT_REVERSED + LAYOUT_STREAMED - d->layout;
        }
        d->t += nsteps;
        if (d->avg_track) d->avg_count += nsteps;
        d->monitored = true;
        d->mon_blocks = (int)((d->n + b->cfg.block - 1) / b->cfg.block);
    }
}

// Each group runs all nsteps before the next group starts (the groups are
// independent), so a group's populations stay in cache between its steps.
int run_steps(lbm_batch* b, int nsteps) {
    if (b->cfg.mode == lbm::BATCH_MODE_INPLACE && (batch_kind(b) & lbm::BATCH_CURVED))
        return fail(LBM_EINVAL, "in-place batch stepping takes no curved walls");
    int rc = refresh_tables(b);
    if (rc) return rc;
    if (nsteps >= GRAPH_STEPS) {
        rc = ensure_graphs(b);
        if (rc) return rc;
    }
    const int ng = (int)b->group_first.size() - 1;
    for (int g = 0; g < ng; ++g) {
        int left = nsteps;
        while (left >= GRAPH_STEPS) {
            HIP_TRY(hipGraphLaunch(b->graphs[g], b->stream), "graph launch");
            left -= GRAPH_STEPS;
        }
        if (left > 0) {
            rc = enqueue_steps(b, g, left);
            if (rc) return rc;
        }
    }
    advance_domains(b, nsteps);
    return LBM_OK;
}

bool valid_config(const lbm_batch* b, const lbm::BatchConfig& c) {
    if (c.mode < lbm::BATCH_MODE_STEP || c.mode > lbm::BATCH_MODE_INPLACE) return false;
    if (c.block != 128 && c.block != 256 && c.block != 512) return false;
    if (c.stream_store != 0 && c.stream_store != 1) return false;
    if (c.stream_store && b->storage >= LBM_F16S) return false;
    if (c.mode == lbm::BATCH_MODE_INPLACE && (c.block != 256 || c.stream_store)) return false;
    return c.grid >= 0 && c.group_mb >= 0;
}

// Tuned configurations of this process, keyed by storage, collision form,
// batch size class and number of domains.
std::mutex g_tune_mutex;
std::map<std::tuple<int, int, int, int>, lbm::BatchConfig> g_tune_cache;

}  // namespace

extern "C" {

int lbm_batch_create(lbm_domain* const* doms, int n, void* hip_stream, lbm_batch** out) {
    if (!out || !doms || n < 1) return fail(LBM_EINVAL, "lbm_batch_create: need at least one domain");
    *out = nullptr;
    for (int k = 0; k < n; ++k) {
        if (!doms[k]) return fail(LBM_EINVAL, "NULL domain in batch");
        if (!doms[k]->dev) return fail(LBM_ESTATE, "every domain needs its device memory attached");
        if (doms[k]->storage != doms[0]->storage) return fail(LBM_EINVAL, "all domains of a batch need the same storage");
        for (int j = 0; j < k; ++j)
            if (doms[j] == doms[k]) return fail(LBM_EINVAL, "a domain appears twice in the batch");
    }
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return fail(LBM_ENOMEM, "host allocation failed");
    b->doms.assign(doms, doms + n);
    b->stream = (hipStream_t)hip_stream;
    b->storage = doms[0]->storage;
    for (lbm_domain* d : b->doms) b->total_nodes += d->n;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    b->off_args = take((size_t)n * sizeof(lbm::StepArgs));
    int64_t max_items = 0;   // work items at the smallest work-group size
    for (lbm_domain* d : b->doms) {
        max_items += (d->n + 127) / 128;
        if ((d->n + 127) / 128 > lbm::ITEM_BLOCK_MASK) {
            delete b;
            return fail(LBM_EINVAL, "domain too large for the batch work-item table");
        }
    }
    if (n > (1 << (31 - lbm::ITEM_DOMAIN_SHIFT))) {
        delete b;
        return fail(LBM_EINVAL, "too many domains in one batch");
    }
    b->off_items = take((size_t)max_items * sizeof(int));
    b->off_barrier = take(lbm::BARRIER_WORDS * sizeof(unsigned));
    b->off_error = take(sizeof(int));
    b->dev_bytes = off;
    *out = b;
    return LBM_OK;
}

int lbm_batch_device_bytes(const lbm_batch* b, size_t* bytes) {
    if (!b || !bytes) return fail(LBM_EINVAL, "NULL argument");
    *bytes = b->dev_bytes;
    return LBM_OK;
}

int lbm_batch_attach_device(lbm_batch* b, void* dev_ptr, size_t bytes) {
    if (!b || !dev_ptr) return fail(LBM_EINVAL, "NULL argument");
    if (bytes < b->dev_bytes) return fail(LBM_ENOMEM, "device buffer smaller than lbm_batch_device_bytes");
    if (((uintptr_t)dev_ptr & 255u) != 0) return fail(LBM_EINVAL, "device buffer must be 256-byte aligned");
    b->dev = (char*)dev_ptr;
    b->built_block = 0;
    b->drop_graph();
    HIP_TRY(lbm::launch_fill_zero(b->dev, b->dev_bytes, b->stream), "clearing batch memory");
    return LBM_OK;
}

int lbm_batch_config(const lbm_batch* b, int cfg[5]) {
    if (!b || !cfg) return fail(LBM_EINVAL, "NULL argument");
    cfg[0] = b->cfg.mode;
    cfg[1] = b->cfg.block;
    cfg[2] = b->cfg.stream_store;
    cfg[3] = b->cfg.grid;
    cfg[4] = b->cfg.group_mb;
    return LBM_OK;
}

int lbm_batch_set_config(lbm_batch* b, const int cfg[5]) {
    if (!b || !cfg) return fail(LBM_EINVAL, "NULL argument");
    const lbm::BatchConfig c{cfg[0], cfg[1], cfg[2], cfg[3], cfg[4]};
    if (!valid_config(b, c)) return fail(LBM_EINVAL, "invalid batch configuration");
    b->cfg = c;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, int nsteps) {
    if (!b) return fail(LBM_EINVAL, "NULL argument");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (!b->dev) return fail(LBM_ESTATE, "no device memory attached to the batch");
    b->rates_one = true;
    for (lbm_domain* d : b->doms) {
        if (!d->initialized) return fail(LBM_ESTATE, "every domain must be initialised");
        b->rates_one = b->rates_one && d->rates_one();
    }
    if (nsteps == 0) return LBM_OK;
    return run_steps(b, nsteps);
}

int lbm_batch_autotune(lbm_batch* b, int trial_steps, double* best_ms_per_step) {
    if (!b) return fail(LBM_EINVAL, "NULL argument");
    if (trial_steps < 1) return fail(LBM_EINVAL, "trial_steps must be >= 1");
    if (!b->dev) return fail(LBM_ESTATE, "no device memory attached to the batch");
    for (lbm_domain* d : b->doms)
        if (!d->initialized) return fail(LBM_ESTATE, "every domain must be initialised");
    b->rates_one = true;
    for (lbm_domain* d : b->doms) b->rates_one = b->rates_one && d->rates_one();
    const auto key = std::make_tuple(b->storage, batch_kind(b), (int)std::lround(std::log2((double)b->total_nodes)),
                                     (int)b->doms.size());
    {
        std::lock_guard<std::mutex> lock(g_tune_mutex);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end() && !best_ms_per_step && valid_config(b, it->second)) {
            b->cfg = it->second;
            return LBM_OK;
        }
    }
    std::vector<lbm::BatchConfig> cands;
    for (int group_mb : {0, 96, 192})
        for (int mode : {0, 1})
            for (int block : {128, 256, 512})
                for (int ns : {0, 1}) {
                    if (ns && b->storage >= LBM_F16S) continue;
                    if (mode == 0) cands.push_back({0, block, ns, 0, group_mb});
                    else {
                        cands.push_back({1, block, ns, 0, group_mb});
                        cands.push_back({1, block, ns, -2, group_mb});   // half of the resident capacity
                    }
                }
    // in place: one buffer per domain, so a group of the same budget holds
    // twice the nodes; the best groups hold about 140-160 MiB of populations
    // (measured), so the budgets step finely there
    if (!(batch_kind(b) & lbm::BATCH_CURVED))
        for (int group_mb : {0, 96, 128, 144, 160, 176, 192})
            cands.push_back({lbm::BATCH_MODE_INPLACE, 256, 0, 0, group_mb});
    const int graphs = std::max(1, (trial_steps + GRAPH_STEPS - 1) / GRAPH_STEPS);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "event create");
    HIP_TRY(hipEventCreate(&e1), "event create");
    double best = 1e300;
    lbm::BatchConfig best_cfg = b->cfg;
    int rc = LBM_OK;
    for (lbm::BatchConfig c : cands) {
        if (c.grid == -2) {
            int cap = 0;
            if (lbm::batch_persistent_capacity(b->storage, batch_kind(b), c, &cap) != hipSuccess || cap < 2) continue;
            c.grid = cap / 2;
        }
        b->cfg = c;
        rc = run_steps(b, GRAPH_STEPS);   // warm-up, builds the graphs and tables
        if (rc) break;
        HIP_TRY(hipEventRecord(e0, b->stream), "event record");
        rc = run_steps(b, graphs * GRAPH_STEPS);
        if (rc) break;
        HIP_TRY(hipEventRecord(e1, b->stream), "event record");
        HIP_TRY(hipEventSynchronize(e1), "event synchronize");
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "event time");
        const double per = ms / (graphs * GRAPH_STEPS);
        if (per < best) {
            best = per;
            best_cfg = c;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc) return rc;
    b->cfg = best_cfg;
    if (best_ms_per_step) *best_ms_per_step = best;
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    g_tune_cache[key] = best_cfg;
    return LBM_OK;
}

int lbm_batch_status(lbm_batch* b) {
    if (!b) return fail(LBM_EINVAL, "NULL argument");
    if (!b->dev) return fail(LBM_ESTATE, "no device memory attached to the batch");
    HIP_TRY(hipMemcpyAsync(&b->error_host, b->dev + b->off_error, sizeof(int), hipMemcpyDeviceToHost, b->stream),
            "batch status copy");
    HIP_TRY(hipStreamSynchronize(b->stream), "stream synchronize");
    if (b->error_host) return fail(LBM_EDEVICE, "a device-wide barrier wait exceeded its bound (results invalid)");
    return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) { delete b; }

}  // extern "C"

namespace lbm {

#define LBM_BATCH_SWITCH(FN, ...)                                                     \
    switch (storage) {                                                                \
        case 0: return FN(storage, __VA_ARGS__, std::integral_constant<int, 0>());    \
        case 1: return FN(storage, __VA_ARGS__, std::integral_constant<int, 1>());    \
        case 2: return FN(storage, __VA_ARGS__, std::integral_constant<int, 2>());    \
        case 3: return FN(storage, __VA_ARGS__, std::integral_constant<int, 3>());    \
        default: return hipErrorInvalidValue;                                         \
    }

hipError_t launch_batch_step(int storage, int kind, const BatchArgs& b, const BatchConfig& c, int step,
                             bool monitor, hipStream_t stream) {
    LBM_BATCH_SWITCH(launch_batch_step_s, kind, b, c, step, monitor, stream)
}

hipError_t launch_batch_persistent(int storage, int kind, const BatchArgs& b, const BatchConfig& c,
                                   int step0, int nsteps, hipStream_t stream) {
    LBM_BATCH_SWITCH(launch_batch_persistent_s, kind, b, c, step0, nsteps, stream)
}

hipError_t batch_persistent_capacity(int storage, int kind, const BatchConfig& c, int* blocks) {
    LBM_BATCH_SWITCH(batch_persistent_capacity_s, kind, c, blocks)
}

#undef LBM_BATCH_SWITCH

}  // namespace lbm
