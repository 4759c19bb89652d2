// C ABI of the lattice Boltzmann library: domain construction from a voxel
// mask, parameter validation, inlet profile coefficients, device-memory
// layout, and the launch sequence of the HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include <algorithm>

#include "lbm.h"
#include "lbm_host.h"
#include "lbm_internal.h"

using lbm::SpecialNode;

namespace lbm_host {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace lbm_host

using namespace lbm_host;

namespace {

constexpr int ROW_TILE = 8;   // default rows per tile side in the list order

size_t storage_bytes(int storage) {
    switch (storage) {
        case LBM_F64: return 8;
        case LBM_F32: return 4;
        case LBM_F16S: return 2;
        case LBM_BF16S: return 2;
        default: return 0;
    }
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Complex Bessel function J0 by its power series sum_k (-z^2/4)^k / (k!)^2
// (converges for every z; the arguments here have |z| < 10).
std::complex<double> bessel_j0(std::complex<double> z) {
    const std::complex<double> q = -z * z / 4.0;
    std::complex<double> term = 1.0, sum = 1.0;
    for (int k = 1; k < 300; ++k) {
        term *= q / (double(k) * double(k));
        sum += term;
        if (std::abs(term) < 1e-18 * std::abs(sum)) break;
    }
    return sum;
}

// Steady part a0 and complex oscillating amplitude a1 of the Womersley speed
// U(r, t) = a0 + Re(a1 e^{i omega t}) in a pipe of radius R.
void womersley_coeffs(double r, double R, double nu, double G0, double G1, double omega,
                      double* a0, std::complex<double>* a1) {
    *a0 = 0.0;
    *a1 = 0.0;
    if (!(r < R)) return;
    *a0 = G0 * (R * R - r * r) / (4.0 * nu);
    if (omega != 0.0 && G1 != 0.0) {
        const double alpha = R * std::sqrt(omega / nu);
        const std::complex<double> i32 = std::polar(1.0, 0.75 * M_PI);   // i^{3/2}
        const std::complex<double> ratio = bessel_j0(i32 * (alpha * r / R)) / bessel_j0(i32 * alpha);
        *a1 = G1 / (std::complex<double>(0.0, 1.0) * omega) * (1.0 - ratio);
    }
}

}  // namespace

namespace lbm_host {

bool finite_all(const double* v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

}  // namespace lbm_host


namespace lbm_host {

lbm::StepArgs make_args(const lbm_domain* d) {
    lbm::StepArgs a{};
    char* base = d->dev;
    const bool in_a = (d->cur ^ d->pop_flip) == 0;
    char* in = base + (in_a ? d->off_popA : d->off_popB);
    a.fin = in;
    // in-place streaming reads and writes one buffer
    a.fout = d->layout != LAYOUT_PULL ? in : base + (in_a ? d->off_popB : d->off_popA);
    a.node = (const uint32_t*)(base + d->off_node);
    a.wave_special = (const uint32_t*)(base + d->off_wspec);
    a.rowtab = (const lbm::RowEntry*)(base + d->off_rowtab);
    a.spec = (const SpecialNode*)(base + d->off_spec);
    a.link_meta = (const int32_t*)(base + d->off_lmeta);
    a.link_coef = (const double*)(base + d->off_lcoef);
    a.link_add = (double*)(base + d->off_ladd);
    a.crec = d->crec.empty() ? nullptr : base + d->off_crec;
    a.cside = d->crec.empty() ? nullptr : base + d->off_cside;
    a.crec_base = (const uint32_t*)(base + d->off_cbase);
    a.tcount = (int64_t*)(base + d->off_tcount);
    a.trig = (double*)(base + d->off_trig);
    a.cos_w = std::cos(d->omega);
    a.sin_w = std::sin(d->omega);
    a.partials = (double*)(base + d->off_part);
    a.avg = d->avg_track ? (double*)(base + d->off_avg) : nullptr;
    a.probe_node = (const int32_t*)(base + d->off_probe);
    a.probe_out = d->probe_out;
    a.probe_t0 = d->probe_t0;
    a.probe_cap = d->probe_cap;
    a.nprobe = d->nprobe;
    a.probe_every = d->probe_every;
    a.tin = d->cur;
    a.collision = d->collision;
    a.n = (int)d->n;
    a.npad = d->npad;
    a.nx = d->nx;
    a.ny = d->ny;
    a.nz = d->nz;
    a.W = d->W;
    a.periodic = (int)d->periodic;
    a.nblocks = d->nblocks;
    a.blocks_per_xcd = d->blocks_per_xcd;
    a.s[0] = 1.0 / d->tau;
    for (int k = 0; k < 4; ++k) a.s[k + 1] = d->s[k];
    for (int k = 0; k < 3; ++k) a.g[k] = d->g[k];
    a.omega = d->omega;
    const double an = std::sqrt(d->axis[0] * d->axis[0] + d->axis[1] * d->axis[1] + d->axis[2] * d->axis[2]);
    for (int k = 0; k < 3; ++k) a.axis[k] = an > 0 ? d->axis[k] / an : 0.0;
    a.rho_out = d->rho_out;
    return a;
}

}  // namespace lbm_host

namespace {

// Exact odd polynomial of the moving-wall term f_eq_a(1, axis U) - f_eq_abar(1, axis U)
// in the speed U: the product form of the equilibrium is prod_d psi(c_d, axis_d U)
// with psi(0, v) = 2/3 - v^2 and psi(+-1, v) = (1/3 + v^2 +- v)/2; reversing c
// flips the odd coefficients, so the difference is twice the odd part.
void moving_wall_poly(int a, const double ax[3], double k[3]) {
    const int c[3] = {a % 3 - 1, (a / 3) % 3 - 1, a / 9 - 1};
    double P[7] = {1, 0, 0, 0, 0, 0, 0};
    for (int d = 0; d < 3; ++d) {
        const double p0 = c[d] == 0 ? 2.0 / 3.0 : 1.0 / 6.0;
        const double p1 = c[d] == 0 ? 0.0 : 0.5 * c[d] * ax[d];
        const double p2 = c[d] == 0 ? -ax[d] * ax[d] : 0.5 * ax[d] * ax[d];
        double Q[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int i = 0; i < 5; ++i) {
            Q[i] += P[i] * p0;
            Q[i + 1] += P[i] * p1;
            Q[i + 2] += P[i] * p2;
        }
        std::memcpy(P, Q, sizeof P);
    }
    k[0] = 2.0 * P[1];
    k[1] = 2.0 * P[3];
    k[2] = 2.0 * P[5];
}

// Inlet phase slots for time t: slot t & 1 holds (cos, sin)(omega t), slot
// (t + 1) & 1 the next time.
int upload_phase(lbm_domain* d, int64_t t) {
    for (int q = 0; q < 2; ++q) {
        const int64_t tt = t + q;
        const double ph = d->omega * (double)tt;
        d->trig_host[2 * (tt & 1)] = std::cos(ph);
        d->trig_host[2 * (tt & 1) + 1] = std::sin(ph);
    }
    HIP_TRY(hipMemcpyAsync(d->dev + d->off_trig, d->trig_host, sizeof d->trig_host, hipMemcpyHostToDevice, d->stream),
            "upload of the inlet phase");
    return LBM_OK;
}

}  // namespace

namespace lbm_host {

// Recompute the inlet coefficients (they depend on tau through nu) and upload
// them with the inlet phase of the current time.
int prepare_links(lbm_domain* d) {
    if (!d->links_dirty) return LBM_OK;
    if (d->nlinks() == 0) {
        d->links_dirty = false;
        return LBM_OK;
    }
    if (d->has_inlet_links && !d->inlet_set)
        return fail(LBM_ESTATE, "the mask has inlet cells: call lbm_set_inlet_womersley first");
    const double nu = (d->tau - 0.5) / 3.0;
    const double an = std::sqrt(d->axis[0] * d->axis[0] + d->axis[1] * d->axis[1] + d->axis[2] * d->axis[2]);
    const double ax[3] = {d->axis[0] / an, d->axis[1] / an, d->axis[2] / an};
    for (size_t k = 0; k < d->nlinks(); ++k) {
        double* cf = &d->link_coef[lbm::LINK_COEFS * k];
        for (int q = 0; q < lbm::LINK_COEFS; ++q) cf[q] = 0.0;
        if ((d->link_meta[k] & 0xff) != lbm::LINK_INLET) continue;
        const int a = d->link_meta[k] >> 8;
        const int c[3] = {a % 3 - 1, (a / 3) % 3 - 1, a / 9 - 1};
        const int32_t* p = &d->link_xyz[3 * k];
        // link midpoint between the node and its source x - c_alpha
        const double m[3] = {p[0] - 0.5 * c[0], p[1] - 0.5 * c[1], p[2] - 0.5 * c[2]};
        double dv[3], along = 0.0;
        for (int q = 0; q < 3; ++q) {
            dv[q] = m[q] - d->center[q];
            along += dv[q] * ax[q];
        }
        double r2 = 0.0;
        for (int q = 0; q < 3; ++q) {
            const double e = dv[q] - along * ax[q];
            r2 += e * e;
        }
        double a0;
        std::complex<double> a1;
        womersley_coeffs(std::sqrt(r2), d->radius, nu, d->G0, d->G1, d->omega, &a0, &a1);
        cf[0] = a0;
        cf[1] = a1.real();
        cf[2] = a1.imag();
        moving_wall_poly(a, ax, cf + 3);
    }
    if (d->dev) {
        HIP_TRY(hipMemcpyAsync(d->dev + d->off_lcoef, d->link_coef.data(), d->link_coef.size() * sizeof(double),
                               hipMemcpyHostToDevice, d->stream),
                "upload of boundary links");
        int rc = upload_phase(d, d->t);
        if (rc) return rc;
        d->links_dirty = false;
    }
    return LBM_OK;
}

}  // namespace lbm_host

bool lbm_domain::use_inplace() const {
    if (stream_mode == LBM_STREAM_PULL) return false;
    if (stream_mode == LBM_STREAM_INPLACE) return true;
    // curved walls step faster with pull (their in-place kinds need the
    // wall links in both kinds and the own-value records)
    if (!crec.empty()) return false;
    // 4- and 8-byte populations whose two pull buffers no longer stay in the
    // Infinity Cache, while one buffer is small enough for it to serve part
    // of the in-place traffic
    return storage_bytes(storage) >= 4 && 2 * pop_bytes > lbm_host::STREAM_STORE_BYTES &&
           pop_bytes <= lbm_host::INPLACE_MAX_BYTES;
}

namespace lbm_host {

int sync_pull(lbm_domain* d) {
    if (d->layout == LAYOUT_PULL) return LBM_OK;
    lbm::StepArgs a = make_args(d);
    if (d->layout == LAYOUT_REVERSED) {
        // slot reversal in place
        HIP_TRY(lbm::launch_inplace_reverse(d->storage, a, false, d->stream), "in-place layout");
    } else {
        // the streamed layout is a permutation of the post-collision values:
        // gathered into the other buffer, which becomes the one read next
        const bool in_a = (d->cur ^ d->pop_flip) == 0;
        a.fout = d->dev + (in_a ? d->off_popB : d->off_popA);
        HIP_TRY(lbm::launch_inplace_unstream(d->storage, a, d->stream), "in-place layout");
        d->pop_flip ^= 1;
    }
    d->layout = LAYOUT_PULL;
    return LBM_OK;
}

int enter_inplace(lbm_domain* d) {
    const lbm::StepArgs a = make_args(d);
    // curved walls: the blend's own values start from the pull layout
    HIP_TRY(lbm::launch_inplace_reverse(d->storage, a, !d->crec.empty(), d->stream), "in-place layout");
    d->layout = LAYOUT_REVERSED;
    return LBM_OK;
}

}  // namespace lbm_host

namespace {

// Launch nsteps steps; the last one accumulates the monitors.
// The bookkeeping of one step: the next time slot; an in-place step stays on
// its buffer and turns the layout (reversed <-> streamed).
void advance_state(lbm_domain* d) {
    d->cur ^= 1;
    if (d->layout != LAYOUT_PULL) {
        d->pop_flip ^= 1;
        d->layout = LAYOUT_REVERSED + LAYOUT_STREAMED - d->layout;
    }
}

int launch_steps_eager(lbm_domain* d, int nsteps) {
    const bool big = 2 * d->pop_bytes > lbm_host::STREAM_STORE_BYTES;
    for (int k = 0; k < nsteps; ++k) {
        lbm::StepArgs a = make_args(d);
        const int ip = d->layout == LAYOUT_REVERSED   ? lbm::STREAM_NEIGHBOUR
                       : d->layout == LAYOUT_STREAMED ? lbm::STREAM_LOCAL
                                                      : lbm::STREAM_PULL;
        const lbm::StepVariant v{k == nsteps - 1, d->rates_one(), d->periodic_yz(), big && ip == lbm::STREAM_PULL,
                                 d->collision == 1, !d->crec.empty(), ip};
        HIP_TRY(lbm::launch_step(d->storage, a, v, d->stream), "step kernel");
        advance_state(d);
    }
    return LBM_OK;
}

// Capture GRAPH_STEPS steps starting from the current state into a graph.
int build_graph(lbm_domain* d) {
    const int cur = d->cur, flip = d->pop_flip, layout = d->layout, key = d->graph_key();
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(d->stream, hipStreamCaptureModeRelaxed), "graph capture begin");
    int rc = launch_steps_eager(d, GRAPH_STEPS);
    hipError_t e = hipStreamEndCapture(d->stream, &g);
    // nothing ran during capture
    d->cur = cur;
    d->pop_flip = flip;
    d->layout = layout;
    if (rc) {
        if (g) hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "graph capture end");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "graph instantiate");
    d->graph[key] = ex;
    return LBM_OK;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return g_last_error.c_str(); }

int lbm_inlet_profile(double r, double t, double radius, double nu, double G0, double G1, double omega,
                      double* speed) {
    if (!speed || !(radius > 0) || !(nu > 0) || !std::isfinite(r) || !std::isfinite(t))
        return fail(LBM_EINVAL, "lbm_inlet_profile: invalid argument");
    double a0;
    std::complex<double> a1;
    womersley_coeffs(r, radius, nu, G0, G1, omega, &a0, &a1);
    *speed = a0 + a1.real() * std::cos(omega * t) - a1.imag() * std::sin(omega * t);
    return LBM_OK;
}

}  // extern "C"

namespace {

// Curved-wall distances keyed by (cell * 27 + alpha_in): alpha_in is the
// incoming direction of the link, whose source x - c_alpha_in is the wall.
using WallQ = std::unordered_map<int64_t, double>;

int create_domain(const uint8_t* mask, int nx, int ny, int nz, unsigned periodic_bits, int storage,
                  void* hip_stream, const WallQ* wq, int row_tile, lbm_domain** out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mask) return fail(LBM_EINVAL, "mask is NULL");
    if (nx < 1 || ny < 1 || nz < 1 || nx > lbm::MAX_DIM || ny > lbm::MAX_DIM || nz > lbm::MAX_DIM)
        return fail(LBM_EINVAL, "dimensions must be in [1, 1023]");
    if (periodic_bits > 7) return fail(LBM_EINVAL, "periodic_bits must be a combination of LBM_PERIODIC_*");
    if (storage_bytes(storage) == 0) return fail(LBM_EINVAL, "unknown storage type");
    const int64_t cells = (int64_t)nx * ny * nz;
    int64_t nfluid = 0;
    for (int64_t c = 0; c < cells; ++c) {
        if (mask[c] > LBM_OUTLET) return fail(LBM_EINVAL, "mask values must be 0..3");
        nfluid += mask[c] == LBM_FLUID;
    }
    if (nfluid == 0) return fail(LBM_EINVAL, "the mask has no fluid cell");
    const int64_t npad = (nfluid + lbm::BLOCK - 1) / lbm::BLOCK * lbm::BLOCK;
    if (npad * 27 * (int64_t)storage_bytes(storage) >= ((int64_t)1 << 32))
        return fail(LBM_EINVAL, "too many fluid nodes for 32-bit byte offsets");

    lbm_domain* d = new (std::nothrow) lbm_domain();
    if (!d) return fail(LBM_ENOMEM, "host allocation failed");
    try {
        d->nx = nx;
        d->ny = ny;
        d->nz = nz;
        d->periodic = periodic_bits;
        d->storage = storage;
        d->stream = (hipStream_t)hip_stream;
        d->n = nfluid;
        d->npad = (int)npad;
        d->W = (nx + lbm::ROW_SPAN - 1) / lbm::ROW_SPAN;
        d->row_tile = row_tile;
        d->rows = (ny + 2) * (nz + 2);
        d->nblocks = (int)(npad / lbm::BLOCK);
        d->blocks_per_xcd = (d->nblocks + 7) / 8;

        // row table: overlapping fluid bitmaps of each row (one empty row ring
        // around the box) and the list index of each entry's first cell
        d->rowtab.assign((size_t)d->rows * d->W, lbm::RowEntry{0u, 0});
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y) {
                const size_t r = (size_t)d->row_of(y, z) * d->W;
                for (int x = 0; x < nx; ++x) {
                    if (mask[d->cell(x, y, z)] != LBM_FLUID) continue;
                    const int k = (x + 1) / lbm::ROW_SPAN, j = x + 1 - k * lbm::ROW_SPAN;
                    if (k < d->W) d->rowtab[r + k].bits |= 1u << j;
                    if (j <= 1 && k >= 1) d->rowtab[r + k - 1].bits |= 1u << (j + lbm::ROW_SPAN);
                }
            }
        // List order: rows grouped in tiles of row_tile x row_tile rows of the
        // (y, z) plane, x fastest inside a row.  Neighbouring rows then sit close
        // together in the list, so the lines a wave gathers from are shared by
        // waves that run at nearly the same time.
        std::vector<int> order;
        order.reserve((size_t)ny * nz);
        for (int tz = 0; tz < nz; tz += row_tile)
            for (int ty = 0; ty < ny; ty += row_tile)
                for (int z = tz; z < std::min(nz, tz + row_tile); ++z)
                    for (int y = ty; y < std::min(ny, ty + row_tile); ++y) order.push_back(d->row_of(y, z));
        int64_t cnt = 0;
        for (int r : order) {
            const int z = r / (ny + 2) - 1, y = r % (ny + 2) - 1;
            int x = 0;
            for (int k = 0; k < d->W; ++k) {
                for (; x < std::min(nx, k * lbm::ROW_SPAN - 1); ++x) cnt += mask[d->cell(x, y, z)] == LBM_FLUID;
                d->rowtab[(size_t)r * d->W + k].prefix = (int32_t)cnt;
            }
            for (; x < nx; ++x) cnt += mask[d->cell(x, y, z)] == LBM_FLUID;
        }
        if (cnt != nfluid) return fail(LBM_EINVAL, "internal: bitmap count mismatch");
        if ((int64_t)d->rows * d->W >= ((int64_t)1 << 29)) return fail(LBM_EINVAL, "box too large for the row table");

        d->node_words.assign((size_t)npad, 0u);
        d->coords.resize((size_t)nfluid * 3);
        const int dims[3] = {nx, ny, nz};
        const bool per[3] = {(periodic_bits & 1) != 0, (periodic_bits & 2) != 0, (periodic_bits & 4) != 0};
        const bool per_yz = per[1] || per[2];
        int64_t i = 0;
        // curved walls: per ordinary node, its wall links (bit alpha) and the
        // offset of its weights in cw (in increasing alpha)
        std::vector<uint32_t> node_fw;
        std::vector<int64_t> cw_off;
        std::vector<double> cw;
        if (wq) {
            node_fw.assign((size_t)npad, 0u);
            cw_off.assign((size_t)npad, 0);
        }
        // Curved-wall link of node i at (x, y, z), incoming direction a, abar =
        // 26 - a towards the wall (Eq. (9)-(10), linear interpolation):
        //   q <  1/2: 2q f*_abar(x) + (1 - 2q) f*_abar(x + c_a)
        //   q >= 1/2: f*_abar(x) / 2q + (2q - 1) / 2q f*_a(x)
        // where x + c_a (the node behind x) must be fluid, else the link keeps
        // halfway bounce-back (weights 1, 0).  Returns the weights and the
        // plane and node of the second value.
        auto curved_weights = [&](int x, int y, int z, int64_t node, int a, double& w0, double& w1,
                                  int64_t& node2, int& plane2) {
            const double q = wq->at(d->cell(x, y, z) * 27 + a);
            w0 = 1.0;
            w1 = 0.0;
            node2 = node;
            plane2 = 26 - a;
            if (q >= 0.5) {
                w0 = 1.0 / (2.0 * q);
                w1 = (2.0 * q - 1.0) / (2.0 * q);
                plane2 = a;
                return;
            }
            const int c[3] = {a % 3 - 1, (a / 3) % 3 - 1, a / 9 - 1};
            int b[3] = {x + c[0], y + c[1], z + c[2]};
            bool in = true;
            for (int ax = 0; ax < 3; ++ax) {
                if (b[ax] < 0 || b[ax] >= dims[ax]) {
                    if (per[ax]) b[ax] = (b[ax] + dims[ax]) % dims[ax];
                    else in = false;
                }
            }
            if (in && mask[d->cell(b[0], b[1], b[2])] == LBM_FLUID) {
                w0 = 2.0 * q;
                w1 = 1.0 - 2.0 * q;
                node2 = d->index_of(b[0], b[1], b[2]);
            }
        };
        for (int r : order) {
            const int z = r / (ny + 2) - 1, y = r % (ny + 2) - 1;
            for (int x = 0; x < nx; ++x) {
                    if (mask[d->cell(x, y, z)] != LBM_FLUID) continue;
                    d->coords[3 * i] = x;
                    d->coords[3 * i + 1] = y;
                    d->coords[3 * i + 2] = z;
                    // classify the 27 sources x - c_alpha
                    int kind[27], sx[27], sy[27], sz[27];
                    bool special = false;
                    uint32_t curved = 0;   // incoming directions with a wall distance
                    for (int a = 0; a < 27; ++a) {
                        const int c[3] = {a % 3 - 1, (a / 3) % 3 - 1, a / 9 - 1};
                        int q[3] = {x - c[0], y - c[1], z - c[2]};
                        bool inside = true, xwrap = false;
                        for (int ax = 0; ax < 3; ++ax) {
                            if (q[ax] < 0 || q[ax] >= dims[ax]) {
                                if (per[ax]) {
                                    q[ax] = (q[ax] + dims[ax]) % dims[ax];
                                    if (ax == 0) xwrap = true;
                                } else {
                                    inside = false;
                                }
                            }
                        }
                        kind[a] = inside ? mask[d->cell(q[0], q[1], q[2])] : LBM_SOLID;
                        sx[a] = q[0];
                        sy[a] = q[1];
                        sz[a] = q[2];
                        if (kind[a] == LBM_INLET || kind[a] == LBM_OUTLET) special = true;
                        if (xwrap && kind[a] == LBM_FLUID) special = true;
                        if (wq && kind[a] == LBM_SOLID && wq->count(d->cell(x, y, z) * 27 + a)) curved |= 1u << a;
                    }
                    if (d->index_of(x, y, z) != i) return fail(LBM_EINVAL, "internal: index mismatch");
                    if (wq) {
                        // one signed weight per wall link, in increasing alpha
                        // (halfway links 1; curved: w0, negative for q >= 1/2)
                        uint32_t fw = 0;
                        cw_off[i] = (int64_t)cw.size();
                        for (int a = 0; a < 27; ++a) {
                            if (kind[a] != LBM_SOLID) continue;
                            fw |= 1u << a;
                            double r = 1.0;
                            if ((curved >> a) & 1u) {
                                double w0, w1;
                                int64_t node2;
                                int plane2;
                                curved_weights(x, y, z, i, a, w0, w1, node2, plane2);
                                r = plane2 == a ? -w0 : w0;
                            }
                            cw.push_back(r);
                        }
                        node_fw[i] = fw;
                    }
                    if (!special) {
                        d->node_words[i] = per_yz ? ((uint32_t)x | ((uint32_t)y << 10) | ((uint32_t)z << 20))
                                                  : ((uint32_t)x | ((uint32_t)d->row_of(y, z) << 10));
                    } else {
                        SpecialNode sp{};
                        sp.node = (int32_t)i;
                        sp.link0 = (int32_t)d->nlinks();
                        const int sidx = (int)d->spec.size();
                        for (int a = 0; a < 27; ++a) {
                            // element index and plane of the pulled value; turned into
                            // byte offsets once the storage size is applied below
                            if (kind[a] == LBM_FLUID) {
                                sp.off[a] = (uint32_t)d->index_of(sx[a], sy[a], sz[a]);
                                d->spec_plane.push_back(a);
                            } else {
                                sp.off[a] = (uint32_t)i;
                                d->spec_plane.push_back(26 - a);
                                if (kind[a] == LBM_SOLID) {
                                    sp.wallmask |= 1u << a;
                                } else {
                                    const int32_t type = kind[a] == LBM_INLET ? lbm::LINK_INLET : lbm::LINK_OUTLET;
                                    if (type == lbm::LINK_INLET) d->has_inlet_links = true;
                                    sp.linkmask |= 1u << a;
                                    d->link_meta.push_back(type | (a << 8));
                                    d->link_xyz.push_back(x);
                                    d->link_xyz.push_back(y);
                                    d->link_xyz.push_back(z);
                                    for (int q = 0; q < lbm::LINK_COEFS; ++q) d->link_coef.push_back(0.0);
                                }
                            }
                        }
                        d->spec.push_back(sp);
                        d->node_words[i] = lbm::SPECIAL_BIT | (uint32_t)sidx;
                    }
                    ++i;
            }
        }

        // curved-wall records in the step's order: per 64-node chunk (one
        // wavefront), per incoming direction, per node
        if (wq && !cw.empty()) {
            const int64_t chunks = npad / lbm::CREC_CHUNK;
            d->crec_base.assign((size_t)chunks, 0u);
            d->crec.reserve(cw.size());
            for (int64_t c = 0; c < chunks; ++c) {
                d->crec_base[(size_t)c] = (uint32_t)d->crec.size();
                const int64_t i0 = c * lbm::CREC_CHUNK, i1 = std::min<int64_t>(nfluid, i0 + lbm::CREC_CHUNK);
                for (int a = 0; a < 27; ++a)
                    for (int64_t k = i0; k < i1; ++k) {
                        const uint32_t fw = node_fw[(size_t)k];
                        if ((fw >> a) & 1u)
                            d->crec.push_back(cw[(size_t)(cw_off[(size_t)k] + __builtin_popcount(fw & ((1u << a) - 1u)))]);
                    }
            }
            if (d->crec.size() != cw.size()) return fail(LBM_EINVAL, "internal: curved-wall record count mismatch");
            if (d->crec.size() >= ((size_t)1 << 31)) return fail(LBM_EINVAL, "too many wall links");
            // the arithmetic type of the 2- and 4-byte storage forms
            if (storage != LBM_F64) d->crec_f32.assign(d->crec.begin(), d->crec.end());
        }

        // device layout
        const size_t sb = storage_bytes(storage);
        size_t off = 0;
        auto take = [&](size_t bytes) {
            const size_t o = off;
            off += align256(bytes);
            return o;
        };
        d->pop_bytes = (size_t)27 * npad * sb;
        for (size_t k = 0; k < d->spec.size(); ++k)
            for (int a = 0; a < 27; ++a) {
                const uint64_t byte = (uint64_t)lbm::pop_index(d->spec[k].off[a], (uint32_t)d->spec_plane[27 * k + a], (uint32_t)npad, (uint32_t)sb) * sb;
                d->spec[k].off[a] = (uint32_t)byte;
            }
        d->spec_plane.clear();
        d->spec_plane.shrink_to_fit();
        d->off_popA = take(d->pop_bytes);
        d->off_popB = take(d->pop_bytes);
        d->off_node = take((size_t)npad * 4);
        d->wave_special.assign((size_t)npad / 64, 0u);
        for (int64_t k = 0; k < npad; ++k)
            if (d->node_words[(size_t)k] & lbm::SPECIAL_BIT) d->wave_special[(size_t)(k / 64)] = 1u;
        d->off_wspec = take(d->wave_special.size() * 4);
        d->off_rowtab = take(d->rowtab.size() * sizeof(lbm::RowEntry) + 16);
        d->off_spec = take(std::max<size_t>(1, d->spec.size()) * sizeof(SpecialNode));
        const size_t nl = std::max<size_t>(1, d->nlinks());
        d->off_lmeta = take(nl * sizeof(int32_t));
        d->off_lcoef = take(nl * lbm::LINK_COEFS * sizeof(double));
        d->off_ladd = take(nl * sizeof(double));
        d->off_tcount = take(2 * sizeof(int64_t));
        d->off_trig = take(4 * sizeof(double));
        // monitor partials: one per work-group, for work-groups down to 64 nodes
        d->off_part = take((size_t)(npad / 64 + 1) * lbm::MON_WORDS * sizeof(double));
        d->off_monout = take(lbm::MON_WORDS * sizeof(double));
        d->off_avg = take((size_t)3 * nfluid * sizeof(double));
        d->off_probe = take(lbm::MAX_PROBES * sizeof(int32_t));
        d->off_crec = take(std::max<size_t>(1, d->crec.size()) * (storage == LBM_F64 ? 8 : 4));
        d->off_cbase = take(std::max<size_t>(1, d->crec_base.size()) * sizeof(uint32_t));
        // curved walls streamed in place: the own value of each wall link
        d->off_cside = take(std::max<size_t>(1, d->crec.size()) * sb);
        d->dev_bytes = off;
    } catch (const std::bad_alloc&) {
        delete d;
        return fail(LBM_ENOMEM, "host allocation failed");
    }
    *out = d;
    return LBM_OK;
}

// Cell beyond (x, y, z) along c_alpha with periodic wrap, or -1 outside a
// non-periodic box.
int64_t neighbour_cell(int x, int y, int z, int alpha, int nx, int ny, int nz, unsigned periodic_bits) {
    int p[3] = {x + alpha % 3 - 1, y + (alpha / 3) % 3 - 1, z + alpha / 9 - 1};
    const int dims[3] = {nx, ny, nz};
    for (int ax = 0; ax < 3; ++ax) {
        if (p[ax] >= 0 && p[ax] < dims[ax]) continue;
        if (!((periodic_bits >> ax) & 1u)) return -1;
        p[ax] = (p[ax] + dims[ax]) % dims[ax];
    }
    return ((int64_t)p[2] * ny + p[1]) * nx + p[0];
}

}  // namespace

extern "C" {

int lbm_create_domain(const uint8_t* mask, int nx, int ny, int nz, unsigned periodic_bits, int storage,
                      void* hip_stream, lbm_domain** out) {
    return create_domain(mask, nx, ny, nz, periodic_bits, storage, hip_stream, nullptr, ROW_TILE, out);
}

int lbm_wall_links(const uint8_t* mask, int nx, int ny, int nz, unsigned periodic_bits, int32_t* links,
                   int64_t* count) {
    if (!mask || !count) return fail(LBM_EINVAL, "NULL argument");
    if (nx < 1 || ny < 1 || nz < 1 || nx > lbm::MAX_DIM || ny > lbm::MAX_DIM || nz > lbm::MAX_DIM)
        return fail(LBM_EINVAL, "dimensions must be in [1, 1023]");
    if (periodic_bits > 7) return fail(LBM_EINVAL, "periodic_bits must be a combination of LBM_PERIODIC_*");
    int64_t k = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                if (mask[((int64_t)z * ny + y) * nx + x] != LBM_FLUID) continue;
                for (int a = 0; a < 27; ++a) {
                    if (a == 13) continue;
                    const int64_t nb = neighbour_cell(x, y, z, a, nx, ny, nz, periodic_bits);
                    if (nb >= 0 && mask[nb] != LBM_SOLID) continue;
                    if (links) {
                        links[4 * k] = x;
                        links[4 * k + 1] = y;
                        links[4 * k + 2] = z;
                        links[4 * k + 3] = a;
                    }
                    ++k;
                }
            }
    *count = k;
    return LBM_OK;
}

}  // extern "C"

namespace {

// Validate the curved-wall links of lbm_create_domain_curved and key their
// distances by (cell * 27 + incoming direction).
int wall_q_from_links(const uint8_t* mask, int nx, int ny, int nz, unsigned periodic_bits, const int32_t* links,
                      const double* q, int64_t nwall, WallQ& wq) {
    if (!mask || nwall < 0 || (nwall > 0 && (!links || !q))) return fail(LBM_EINVAL, "NULL argument");
    if (nx < 1 || ny < 1 || nz < 1 || nx > lbm::MAX_DIM || ny > lbm::MAX_DIM || nz > lbm::MAX_DIM)
        return fail(LBM_EINVAL, "dimensions must be in [1, 1023]");
    if (periodic_bits > 7) return fail(LBM_EINVAL, "periodic_bits must be a combination of LBM_PERIODIC_*");
    try {
        wq.reserve((size_t)nwall);
        for (int64_t k = 0; k < nwall; ++k) {
            const int x = links[4 * k], y = links[4 * k + 1], z = links[4 * k + 2], a = links[4 * k + 3];
            if (x < 0 || x >= nx || y < 0 || y >= ny || z < 0 || z >= nz || a < 0 || a > 26 || a == 13)
                return fail(LBM_EINVAL, "wall link out of range");
            const int64_t c = ((int64_t)z * ny + y) * nx + x;
            if (mask[c] != LBM_FLUID) return fail(LBM_EINVAL, "wall link from a cell that is not fluid");
            const int64_t nb = neighbour_cell(x, y, z, a, nx, ny, nz, periodic_bits);
            if (nb >= 0 && mask[nb] != LBM_SOLID) return fail(LBM_EINVAL, "wall link does not end in a solid cell");
            if (!std::isfinite(q[k]) || !(q[k] > 0.0) || !(q[k] <= 1.0))
                return fail(LBM_EINVAL, "wall distance q must be in (0, 1]");
            // keyed by the incoming direction 26 - a of the bounced population
            if (!wq.emplace(c * 27 + (26 - a), q[k]).second) return fail(LBM_EINVAL, "duplicate wall link");
        }
    } catch (const std::bad_alloc&) {
        return fail(LBM_ENOMEM, "host allocation failed");
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_create_domain_curved(const uint8_t* mask, int nx, int ny, int nz, unsigned periodic_bits, int storage,
                             const int32_t* links, const double* q, int64_t nwall, void* hip_stream,
                             lbm_domain** out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    WallQ wq;
    const int rc = wall_q_from_links(mask, nx, ny, nz, periodic_bits, links, q, nwall, wq);
    if (rc) return rc;
    return create_domain(mask, nx, ny, nz, periodic_bits, storage, hip_stream, &wq, ROW_TILE, out);
}

int lbm_create_domain_ex(const uint8_t* mask, int nx, int ny, int nz, unsigned periodic_bits, int storage,
                         const int32_t* links, const double* q, int64_t nwall, int row_tile, void* hip_stream,
                         lbm_domain** out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (row_tile < 1 || row_tile > 32 || (row_tile & (row_tile - 1)) != 0)
        return fail(LBM_EINVAL, "row_tile must be 1, 2, 4, 8, 16 or 32");
    if (nwall == 0 && !links && !q)
        return create_domain(mask, nx, ny, nz, periodic_bits, storage, hip_stream, nullptr, row_tile, out);
    WallQ wq;
    const int rc = wall_q_from_links(mask, nx, ny, nz, periodic_bits, links, q, nwall, wq);
    if (rc) return rc;
    return create_domain(mask, nx, ny, nz, periodic_bits, storage, hip_stream, &wq, row_tile, out);
}

int lbm_device_bytes(const lbm_domain* d, size_t* bytes) {
    if (!d || !bytes) return fail(LBM_EINVAL, "NULL argument");
    *bytes = d->dev_bytes;
    return LBM_OK;
}

int lbm_attach_device(lbm_domain* d, void* dev_ptr, size_t bytes) {
    if (!d || !dev_ptr) return fail(LBM_EINVAL, "NULL argument");
    if (bytes < d->dev_bytes) return fail(LBM_ENOMEM, "device buffer smaller than lbm_device_bytes");
    if (((uintptr_t)dev_ptr & 255u) != 0) return fail(LBM_EINVAL, "device buffer must be 256-byte aligned");
    d->dev = (char*)dev_ptr;
    d->drop_graphs();
    // new memory holds no state: the pull layout until the next initialisation
    d->cur = 0;
    d->pop_flip = 0;
    d->layout = LAYOUT_PULL;
    hipStream_t st = d->stream;
    HIP_TRY(lbm::launch_fill_zero(d->dev, d->dev_bytes, st), "clearing device memory");
    HIP_TRY(hipMemcpyAsync(d->dev + d->off_node, d->node_words.data(), d->node_words.size() * 4,
                           hipMemcpyHostToDevice, st), "upload of node table");
    HIP_TRY(hipMemcpyAsync(d->dev + d->off_wspec, d->wave_special.data(), d->wave_special.size() * 4,
                           hipMemcpyHostToDevice, st), "upload of special-chunk flags");
    HIP_TRY(hipMemcpyAsync(d->dev + d->off_rowtab, d->rowtab.data(), d->rowtab.size() * sizeof(lbm::RowEntry),
                           hipMemcpyHostToDevice, st), "upload of row table");
    if (!d->spec.empty())
        HIP_TRY(hipMemcpyAsync(d->dev + d->off_spec, d->spec.data(), d->spec.size() * sizeof(SpecialNode),
                               hipMemcpyHostToDevice, st), "upload of special nodes");
    if (!d->crec.empty()) {
        if (d->storage == LBM_F64)
            HIP_TRY(hipMemcpyAsync(d->dev + d->off_crec, d->crec.data(), d->crec.size() * sizeof(double),
                                   hipMemcpyHostToDevice, st), "upload of curved-wall weights");
        else
            HIP_TRY(hipMemcpyAsync(d->dev + d->off_crec, d->crec_f32.data(), d->crec_f32.size() * sizeof(float),
                                   hipMemcpyHostToDevice, st), "upload of curved-wall weights");
        HIP_TRY(hipMemcpyAsync(d->dev + d->off_cbase, d->crec_base.data(), d->crec_base.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, st), "upload of curved-wall record index");
    }
    if (d->nlinks()) {
        HIP_TRY(hipMemcpyAsync(d->dev + d->off_lmeta, d->link_meta.data(), d->nlinks() * sizeof(int32_t),
                               hipMemcpyHostToDevice, st), "upload of link table");
    }
    d->links_dirty = true;
    d->initialized = false;
    d->monitored = false;
    return LBM_OK;
}

int lbm_fluid_count(const lbm_domain* d, int64_t* n) {
    if (!d || !n) return fail(LBM_EINVAL, "NULL argument");
    *n = d->n;
    return LBM_OK;
}

int lbm_fluid_coords(const lbm_domain* d, int32_t* xyz) {
    if (!d || !xyz) return fail(LBM_EINVAL, "NULL argument");
    std::memcpy(xyz, d->coords.data(), d->coords.size() * sizeof(int32_t));
    return LBM_OK;
}

int lbm_set_params(lbm_domain* d, const lbm_params* p) {
    if (!d || !p) return fail(LBM_EINVAL, "NULL argument");
    if (p->struct_size != sizeof(lbm_params)) return fail(LBM_EINVAL, "lbm_params.struct_size mismatch");
    if (!std::isfinite(p->tau) || !(p->tau > 0.5)) return fail(LBM_EINVAL, "tau must be finite and > 1/2");
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(p->s[k]) || !(p->s[k] > 0.0) || !(p->s[k] < 2.0))
            return fail(LBM_EINVAL, "relaxation rates must lie in (0, 2)");
    if (!finite_all(p->g, 3)) return fail(LBM_EINVAL, "body force must be finite");
    d->tau = p->tau;
    for (int k = 0; k < 4; ++k) d->s[k] = p->s[k];
    for (int k = 0; k < 3; ++k) d->g[k] = p->g[k];
    d->params_set = true;
    d->links_dirty = true;
    d->drop_graphs();
    return LBM_OK;
}

int lbm_set_inlet_womersley(lbm_domain* d, const double axis[3], const double center[3], double radius,
                            double G0, double G1, double omega) {
    if (!d || !axis || !center) return fail(LBM_EINVAL, "NULL argument");
    if (!finite_all(axis, 3) || !finite_all(center, 3) || !std::isfinite(radius) || !std::isfinite(G0) ||
        !std::isfinite(G1) || !std::isfinite(omega))
        return fail(LBM_EINVAL, "inlet parameters must be finite");
    if (axis[0] == 0.0 && axis[1] == 0.0 && axis[2] == 0.0) return fail(LBM_EINVAL, "inlet axis is zero");
    if (!(radius > 0.0)) return fail(LBM_EINVAL, "inlet radius must be > 0");
    if (omega < 0.0) return fail(LBM_EINVAL, "omega must be >= 0");
    for (int k = 0; k < 3; ++k) {
        d->axis[k] = axis[k];
        d->center[k] = center[k];
    }
    d->radius = radius;
    d->G0 = G0;
    d->G1 = G1;
    d->omega = omega;
    d->inlet_set = true;
    d->links_dirty = true;
    d->drop_graphs();
    return LBM_OK;
}

int lbm_set_outlet_pressure(lbm_domain* d, double rho_out) {
    if (!d) return fail(LBM_EINVAL, "NULL argument");
    if (!std::isfinite(rho_out) || !(rho_out > 0.0)) return fail(LBM_EINVAL, "rho_out must be finite and > 0");
    d->rho_out = rho_out;
    d->drop_graphs();
    return LBM_OK;
}

int lbm_set_collision(lbm_domain* d, int kind) {
    if (!d) return fail(LBM_EINVAL, "NULL argument");
    if (kind != LBM_COLLISION_CHM_MRT && kind != LBM_COLLISION_SRT2) return fail(LBM_EINVAL, "unknown collision kind");
    d->collision = kind;
    d->drop_graphs();
    return LBM_OK;
}

int lbm_set_streaming(lbm_domain* d, int mode) {
    if (!d) return fail(LBM_EINVAL, "NULL argument");
    if (mode != LBM_STREAM_PULL && mode != LBM_STREAM_INPLACE && mode != LBM_STREAM_AUTO)
        return fail(LBM_EINVAL, "unknown streaming mode");
    d->stream_mode = mode;
    // leaving in-place streaming: the pull step reads the pull layout
    if (!d->use_inplace() && d->dev) return sync_pull(d);
    return LBM_OK;
}

int lbm_streaming_in_place(const lbm_domain* d, int* in_place) {
    if (!d || !in_place) return fail(LBM_EINVAL, "NULL argument");
    *in_place = d->use_inplace() ? 1 : 0;
    return LBM_OK;
}

int lbm_init_equilibrium(lbm_domain* d, const double* rho, const double* u) {
    if (!d) return fail(LBM_EINVAL, "NULL argument");
    if (!d->dev) return fail(LBM_ESTATE, "no device memory attached");
    if (!d->params_set) return fail(LBM_ESTATE, "call lbm_set_params first");
    d->t = 0;
    int rc = prepare_links(d);
    if (rc) return rc;
    rc = upload_phase(d, 0);
    if (rc) return rc;
    d->pop_flip = 0;
    d->layout = LAYOUT_PULL;
    d->cur = 1;   // the init kernel writes into the "next" buffer of slot 1, i.e. buffer A
    lbm::StepArgs a = make_args(d);
    a.tin = 0;
    HIP_TRY(lbm::launch_init(d->storage, a, rho, u, d->stream), "init kernel");
    d->cur = 0;
    d->t = 0;
    d->initialized = true;
    d->monitored = false;
    d->avg_count = 0;
    if (d->avg_track) {
        d->avg_track = false;
        d->drop_graphs();
    }
    if (d->nprobe > 0 && d->probe_t0 != 0) {
        d->probe_t0 = 0;   // records restart with the new run
        d->drop_graphs();
    }
    return LBM_OK;
}

int lbm_step(lbm_domain* d, int nsteps) {
    if (!d) return fail(LBM_EINVAL, "NULL argument");
    if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
    if (!d->initialized) return fail(LBM_ESTATE, "call lbm_init_equilibrium first");
    int rc = prepare_links(d);
    if (rc) return rc;
    if (nsteps > 0 && d->use_inplace() && d->layout == LAYOUT_PULL) {
        rc = enter_inplace(d);
        if (rc) return rc;
    }
    // an in-place batch may have left a pull domain in an in-place layout
    if (nsteps > 0 && !d->use_inplace() && d->layout != LAYOUT_PULL) {
        rc = sync_pull(d);
        if (rc) return rc;
    }
    int left = nsteps;
    // Long runs replay captured graphs of GRAPH_STEPS launches (no host launch
    // gaps); the default (NULL) stream cannot be captured and runs eagerly.
    // The graphs of the current state and of the state one step later are
    // captured together, on the first call after a change that dropped them,
    // so a later call (a timed run) never waits for a capture, whatever step
    // parity it starts at.  GRAPH_STEPS is even: a replay ends in the state it
    // started from.
    if (d->stream != nullptr) {
        if (nsteps > 0) {
            const int cur = d->cur, flip = d->pop_flip, layout = d->layout;
            for (int k = 0; k < 2 && rc == 0; ++k) {
                if (k == 1) advance_state(d);
                if (!d->graph[d->graph_key()]) rc = build_graph(d);
            }
            d->cur = cur;
            d->pop_flip = flip;
            d->layout = layout;
            if (rc) return rc;
        }
        while (left >= GRAPH_STEPS) {
            HIP_TRY(hipGraphLaunch(d->graph[d->graph_key()], d->stream), "graph launch");
            left -= GRAPH_STEPS;
        }
    }
    rc = launch_steps_eager(d, left);
    if (rc) return rc;
    d->t += nsteps;
    if (d->avg_track) d->avg_count += nsteps;
    if (nsteps > 0) {
        d->monitored = true;
        d->mon_blocks = d->nblocks;
    }
    return LBM_OK;
}

int lbm_time(const lbm_domain* d, int64_t* t) {
    if (!d || !t) return fail(LBM_EINVAL, "NULL argument");
    *t = d->t;
    return LBM_OK;
}

int lbm_moments(lbm_domain* d, double* rho, double* u) {
    if (!d) return fail(LBM_EINVAL, "NULL argument");
    if (!d->initialized) return fail(LBM_ESTATE, "call lbm_init_equilibrium first");
    if (!rho && !u) return LBM_OK;
    int rc = sync_pull(d);
    if (rc) return rc;
    lbm::StepArgs a = make_args(d);
    HIP_TRY(lbm::launch_moments(d->storage, a, rho, u, nullptr, 0, 0.0, d->stream), "moments kernel");
    return LBM_OK;
}

int lbm_set_probes(lbm_domain* d, const int32_t* xyz, int nprobe, int every, double* out_dev, int64_t capacity) {
    if (!d) return fail(LBM_EINVAL, "NULL argument");
    if (!d->dev) return fail(LBM_ESTATE, "no device memory attached");
    if (nprobe < 0 || nprobe > lbm::MAX_PROBES) return fail(LBM_EINVAL, "nprobe must be in [0, 64]");
    if (nprobe > 0) {
        if (!xyz || !out_dev) return fail(LBM_EINVAL, "NULL argument");
        if (every < 1 || capacity < 1) return fail(LBM_EINVAL, "every and capacity must be >= 1");
        if (((uintptr_t)out_dev & 7u) != 0) return fail(LBM_EINVAL, "out_dev must be 8-byte aligned");
    }
    std::vector<int32_t> node((size_t)std::max(nprobe, 1), 0);
    for (int k = 0; k < nprobe; ++k) {
        const int x = xyz[3 * k], y = xyz[3 * k + 1], z = xyz[3 * k + 2];
        if (x < 0 || x >= d->nx || y < 0 || y >= d->ny || z < 0 || z >= d->nz)
            return fail(LBM_EINVAL, "probe outside the box");
        if (!d->is_fluid(x, y, z)) return fail(LBM_EINVAL, "probe at a cell that is not fluid");
        node[k] = d->index_of(x, y, z);
    }
    if (nprobe > 0)
        HIP_TRY(hipMemcpyAsync(d->dev + d->off_probe, node.data(), (size_t)nprobe * sizeof(int32_t),
                               hipMemcpyHostToDevice, d->stream), "upload of probe nodes");
    // the host vector must outlive the copy
    HIP_TRY(hipStreamSynchronize(d->stream), "probe upload");
    d->nprobe = nprobe;
    d->probe_every = nprobe > 0 ? every : 1;
    d->probe_out = nprobe > 0 ? out_dev : nullptr;
    d->probe_cap = nprobe > 0 ? capacity : 0;
    d->probe_t0 = d->t;
    d->drop_graphs();
    return LBM_OK;
}

int lbm_probe_count(const lbm_domain* d, int64_t* nrec) {
    if (!d || !nrec) return fail(LBM_EINVAL, "NULL argument");
    *nrec = d->nprobe > 0 ? std::min<int64_t>(d->probe_cap, std::max<int64_t>(0, d->t - d->probe_t0) / d->probe_every)
                          : 0;
    return LBM_OK;
}

int lbm_average(lbm_domain* d, int op, double* u_avg) {
    if (!d) return fail(LBM_EINVAL, "NULL argument");
    if (!d->dev) return fail(LBM_ESTATE, "no device memory attached");
    double* acc = (double*)(d->dev + d->off_avg);
    lbm::StepArgs a = make_args(d);
    switch (op) {
        case LBM_AVG_RESET:
            HIP_TRY(lbm::launch_fill_zero(acc, (size_t)3 * d->n * sizeof(double), d->stream), "average reset");
            d->avg_count = 0;
            if (d->avg_track) {
                d->avg_track = false;
                d->drop_graphs();
            }
            return LBM_OK;
        case LBM_AVG_TRACK:
            if (!d->initialized) return fail(LBM_ESTATE, "call lbm_init_equilibrium first");
            if (!d->avg_track) {
                d->avg_track = true;
                d->drop_graphs();
            }
            return LBM_OK;
        case LBM_AVG_ACCUMULATE: {
            if (!d->initialized) return fail(LBM_ESTATE, "call lbm_init_equilibrium first");
            const int rc = sync_pull(d);
            if (rc) return rc;
            a = make_args(d);
            HIP_TRY(lbm::launch_moments(d->storage, a, nullptr, nullptr, acc, 1, 0.0, d->stream), "average accumulate");
            d->avg_count += 1;
            return LBM_OK;
        }
        case LBM_AVG_READ:
            if (!u_avg) return fail(LBM_EINVAL, "u_avg is NULL");
            if (d->avg_count == 0) return fail(LBM_ESTATE, "nothing accumulated");
            HIP_TRY(lbm::launch_moments(d->storage, a, nullptr, u_avg, acc, 2, (double)d->avg_count, d->stream),
                    "average read");
            return LBM_OK;
        default:
            return fail(LBM_EINVAL, "unknown average op");
    }
}

int lbm_monitors(lbm_domain* d, double out[10]) {
    if (!d || !out) return fail(LBM_EINVAL, "NULL argument");
    if (!d->monitored) return fail(LBM_ESTATE, "no step has run since initialisation");
    double* mo = (double*)(d->dev + d->off_monout);
    HIP_TRY(lbm::launch_monitor_finalize((const double*)(d->dev + d->off_part), d->mon_blocks, mo,
                                         d->stream),
            "monitor reduction");
    HIP_TRY(hipMemcpyAsync(d->mon_host, mo, 9 * sizeof(double), hipMemcpyDeviceToHost, d->stream), "monitor copy");
    HIP_TRY(hipStreamSynchronize(d->stream), "stream synchronize");
    out[0] = (double)d->n + d->mon_host[0];
    for (int k = 1; k < 9; ++k) out[k] = d->mon_host[k];
    out[9] = (double)d->t;
    if (!finite_all(out, 10)) return fail(LBM_EUNSTABLE, "non-finite monitor values: the run diverged");
    return LBM_OK;
}

int lbm_read_populations(lbm_domain* d, double* f_dev) {
    if (!d || !f_dev) return fail(LBM_EINVAL, "NULL argument");
    if (!d->initialized) return fail(LBM_ESTATE, "call lbm_init_equilibrium first");
    const int rc = sync_pull(d);
    if (rc) return rc;
    lbm::StepArgs a = make_args(d);
    HIP_TRY(lbm::launch_read_populations(d->storage, a, f_dev, d->stream), "population read");
    return LBM_OK;
}

namespace {
// Version 2: populations in tiles of 256-byte runs for every storage form
// (version 1 kept one plane per direction for the 2-byte forms); the node
// order's row-tile edge and the population tile are recorded and must match.
constexpr uint32_t STATE_VERSION = 2;
struct StateHeader {
    char magic[8];
    uint32_t version, storage;
    int64_t n, nspec, npad, t;   // nspec: number of open-boundary links
    uint64_t pop_bytes;
    uint32_t row_tile, pop_tile; // row-tile edge of the node order; nodes per population tile
};
}  // namespace

int lbm_get_state(lbm_domain* d, void* host, size_t* bytes) {
    if (!d || !bytes) return fail(LBM_EINVAL, "NULL argument");
    const size_t need = sizeof(StateHeader) + d->pop_bytes + d->nlinks() * sizeof(double);
    if (!host) {
        *bytes = need;
        return LBM_OK;
    }
    if (*bytes < need) return fail(LBM_EINVAL, "state buffer too small");
    if (!d->initialized) return fail(LBM_ESTATE, "call lbm_init_equilibrium first");
    // the state is kept in the pull layout
    const int rc = sync_pull(d);
    if (rc) return rc;
    StateHeader h{};
    std::memcpy(h.magic, "LBMSTAT1", 8);
    h.version = STATE_VERSION;
    h.storage = (uint32_t)d->storage;
    h.row_tile = (uint32_t)d->row_tile;
    h.pop_tile = 1u << lbm::pop_tile_shift((uint32_t)storage_bytes(d->storage));
    h.n = d->n;
    h.nspec = (int64_t)d->nlinks();
    h.npad = d->npad;
    h.t = d->t;
    h.pop_bytes = d->pop_bytes;
    char* p = (char*)host;
    std::memcpy(p, &h, sizeof h);
    const size_t cur_off = (d->cur ^ d->pop_flip) == 0 ? d->off_popA : d->off_popB;
    HIP_TRY(hipMemcpyAsync(p + sizeof h, d->dev + cur_off, d->pop_bytes, hipMemcpyDeviceToHost, d->stream),
            "state copy");
    if (d->nlinks())
        HIP_TRY(hipMemcpyAsync(p + sizeof h + d->pop_bytes, d->dev + d->off_ladd, d->nlinks() * sizeof(double),
                               hipMemcpyDeviceToHost, d->stream), "state copy");
    HIP_TRY(hipStreamSynchronize(d->stream), "stream synchronize");
    *bytes = need;
    return LBM_OK;
}

int lbm_set_state(lbm_domain* d, const void* host, size_t bytes) {
    if (!d || !host) return fail(LBM_EINVAL, "NULL argument");
    if (!d->dev) return fail(LBM_ESTATE, "no device memory attached");
    if (!d->params_set) return fail(LBM_ESTATE, "call lbm_set_params first");
    StateHeader h;
    if (bytes < sizeof h) return fail(LBM_EINVAL, "state too short");
    std::memcpy(&h, host, sizeof h);
    const size_t need = sizeof(StateHeader) + d->pop_bytes + d->nlinks() * sizeof(double);
    if (std::memcmp(h.magic, "LBMSTAT1", 8) != 0 || h.version != STATE_VERSION ||
        h.row_tile != (uint32_t)d->row_tile ||
        h.pop_tile != (1u << lbm::pop_tile_shift((uint32_t)storage_bytes(d->storage))) ||
        h.storage != (uint32_t)d->storage ||
        h.n != d->n || h.nspec != (int64_t)d->nlinks() || h.npad != d->npad || h.pop_bytes != d->pop_bytes ||
        h.t < 0 || bytes < need)
        return fail(LBM_EINVAL, "state header does not match this domain");
    int rc = prepare_links(d);
    if (rc) return rc;
    const char* p = (const char*)host;
    d->cur = 0;
    d->pop_flip = 0;
    d->layout = LAYOUT_PULL;
    HIP_TRY(hipMemcpyAsync(d->dev + d->off_popA, p + sizeof h, d->pop_bytes, hipMemcpyHostToDevice, d->stream),
            "state upload");
    if (d->nlinks())
        HIP_TRY(hipMemcpyAsync(d->dev + d->off_ladd, p + sizeof h + d->pop_bytes, d->nlinks() * sizeof(double),
                               hipMemcpyHostToDevice, d->stream), "state upload");
    d->t_upload[0] = h.t;
    d->t_upload[1] = h.t;
    rc = upload_phase(d, h.t);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(d->dev + d->off_tcount, d->t_upload, sizeof d->t_upload, hipMemcpyHostToDevice, d->stream),
            "state upload");
    HIP_TRY(hipStreamSynchronize(d->stream), "stream synchronize");
    d->t = h.t;
    d->initialized = true;
    d->monitored = false;
    return LBM_OK;
}

void lbm_destroy(lbm_domain* d) { delete d; }

}  // extern "C"
