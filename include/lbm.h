/*
 * lbm.h -- C ABI of the MI355X D3Q27 CHM-MRT lattice Boltzmann library.
 *
 * What the library computes: the lattice Boltzmann evolution equation (Eq. (1))
 * with the central Hermite moment multiple-relaxation-time collision (CHM-MRT,
 * Eq. (6)) and the full-expansion equilibrium (Eq. (3) with the sixth-order
 * D3Q27 expansion of Sec. 2.1.3, whose central moments are (rho, 0, ..., 0),
 * Eq. (8)), on a voxelized vessel: halfway bounce-back walls (Eq. (9) at
 * q = 1/2), a velocity inlet and a pressure outlet built from the bounce-back
 * family (Sec. 2.1.2).  One step is one fused pull-scheme kernel over the list
 * of fluid nodes.
 *
 * Conventions for every function:
 *  - Return value: LBM_OK (0) or a negative LBM_E* code.  Nothing throws or
 *    aborts across the ABI; lbm_last_error() returns a message for the last
 *    failure of the calling thread.
 *  - "host" pointers are read or written during the call and may be freed
 *    afterwards.  "device" pointers are GPU global memory that the caller owns
 *    and keeps alive for as long as the library may use them.
 *  - Device memory: the library never allocates GPU memory.  The caller asks
 *    for the size (lbm_device_bytes), allocates it (for example as a torch
 *    uint8 tensor) and attaches it (lbm_attach_device).
 *  - Work is enqueued on the HIP stream given at creation and is asynchronous
 *    unless the function says it synchronizes.
 *  - A domain is not thread-safe; different domains are independent.
 *
 * Units: lattice units (dx = dt = 1), sound speed squared 1/3, kinematic
 * viscosity nu = (tau - 1/2) / 3.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_domain lbm_domain;   /* opaque, library-owned */
typedef struct lbm_batch lbm_batch;     /* opaque, library-owned */

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* invalid argument */
    LBM_ENOMEM = -2,     /* host allocation failed or device buffer too small */
    LBM_EDEVICE = -3,    /* a HIP call failed (message in lbm_last_error) */
    LBM_EUNSTABLE = -4,  /* non-finite monitor values: the run diverged */
    LBM_ESTATE = -5      /* call out of order (e.g. step before attach) */
};

/* Population storage.  Every storage type holds the shifted populations
 * f - w_alpha (rest state = 0).  F64 and F32 compute in their own precision;
 * F16S and BF16S store IEEE half / bfloat16 (round to nearest even, half
 * subnormals kept) and compute in FP32.  Boundary, force and monitor sums
 * are accumulated in FP64 for every storage type. */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16S = 2, LBM_BF16S = 3 };

/* Mask cell types: mask[(z * ny + y) * nx + x]. */
enum { LBM_SOLID = 0, LBM_FLUID = 1, LBM_INLET = 2, LBM_OUTLET = 3 };

/* Periodic axes. */
enum { LBM_PERIODIC_X = 1, LBM_PERIODIC_Y = 2, LBM_PERIODIC_Z = 4 };

/* Collision parameters (Eq. (6), Sec. 2.1.3).  The six second-order central
 * Hermite moments relax with rate 1/tau (tau > 1/2 sets the viscosity); the
 * moments of orders 3, 4, 5 and 6 relax with the free rates s[0..3], each in
 * (0, 2).  g is a constant body acceleration (force density rho g); it enters
 * the velocity with the half-step shift u = (j + rho g / 2) / rho and the
 * first-order central moments after collision are rho g / 2.  struct_size must
 * be sizeof(lbm_params). */
typedef struct {
    uint32_t struct_size;
    double tau;
    double s[4];
    double g[3];
} lbm_params;

/* Message of the last failing call on this thread ("" if none). */
const char* lbm_last_error(void);

/* Build a domain from a voxel mask (host, copied).
 * nx, ny, nz in [1, 1023]; mask values in {SOLID, FLUID, INLET, OUTLET};
 * at least one FLUID cell.  A fluid node x pulls direction alpha from
 * x - c_alpha: from a FLUID cell by streaming, from a SOLID cell or from
 * outside the box on a non-periodic axis by halfway bounce-back, from an
 * INLET ghost by the velocity inlet rule and from an OUTLET ghost by the
 * pressure outlet rule.  periodic_bits: LBM_PERIODIC_* flags.  storage:
 * LBM_F64 / F32 / F16S / BF16S.  hip_stream: hipStream_t (NULL = default).
 * Fluid nodes are numbered row by row, x fastest within a row; the (y, z)
 * rows are taken in tiles of 8 x 8 (tile y fastest, then tile z, and y
 * fastest inside a tile; lbm_create_domain_ex sets another tile edge).
 * lbm_fluid_coords gives the order explicitly.
 * Errors: EINVAL for bad sizes, values or flags; ENOMEM on host allocation. */
int lbm_create_domain(const uint8_t* mask, int nx, int ny, int nz, unsigned periodic_bits,
                      int storage, void* hip_stream, lbm_domain** out);

/* Curved walls by interpolated bounce-back (Sec. 2.1.4, Eq. (9)-(10), the
 * linear interpolation of Bouzidi et al. that the paper cites).  The same as
 * lbm_create_domain, plus wall distances for nwall links: link k is the fluid
 * cell (x, y, z) = links[4k .. 4k+2] and the direction alpha = links[4k+3]
 * (D3Q27 index, not 13) towards a wall, i.e. the cell x + c_alpha is SOLID or
 * lies outside a non-periodic box (lbm_wall_links lists them); q[k] in (0, 1]
 * is the distance from the node to the wall along the link in units of
 * |c_alpha|.  With abar the opposite direction, the population returning to
 * x is
 *   q <  1/2: 2q f*_alpha(x, t) + (1 - 2q) f*_alpha(x - c_alpha, t),
 *   q >= 1/2: f*_alpha(x, t) / (2q) + (2q - 1) / (2q) f*_abar(x, t),
 * both halfway bounce-back at q = 1/2; for q < 1/2 the node x - c_alpha must
 * be fluid, otherwise that link keeps halfway bounce-back.  The wall force of
 * a curved link is (f*_alpha(x, t) + f_abar(x, t + 1)) c_alpha.  Links not
 * listed keep halfway bounce-back.  The arrays are host memory, read during
 * the call.  The step blends each wall link's bounce-back value with its
 * second value after the gather, from one weight per wall link held in device
 * memory (the link count times the size of the arithmetic type: 8 bytes for
 * LBM_F64, 4 otherwise).  Errors: EINVAL for a link that is out
 * of range, does not start at a fluid cell or end at a wall, is listed twice,
 * or has q outside (0, 1]; otherwise as lbm_create_domain. */
int lbm_create_domain_curved(const uint8_t* mask, int nx, int ny, int nz, unsigned periodic_bits,
                             int storage, const int32_t* links, const double* q, int64_t nwall,
                             void* hip_stream, lbm_domain** out);

/* lbm_create_domain with layout options: the (y, z) rows are taken in tiles
 * of row_tile x row_tile (1, 2, 4, 8, 16 or 32; lbm_create_domain and
 * lbm_create_domain_curved use 8), which changes only the node order, never
 * a result; with nwall > 0 the walls are curved as in
 * lbm_create_domain_curved (links and q NULL with nwall 0 give halfway walls).
 * It serves the choice of the list order by timing (batch autotuning).
 * Errors: EINVAL for any other row_tile; otherwise as the two functions it
 * generalizes. */
int lbm_create_domain_ex(const uint8_t* mask, int nx, int ny, int nz, unsigned periodic_bits, int storage,
                         const int32_t* links, const double* q, int64_t nwall, int row_tile, void* hip_stream,
                         lbm_domain** out);

/* Wall links of a mask (same layout and periodic rules as lbm_create_domain):
 * every pair of a FLUID cell and a direction alpha whose cell x + c_alpha is
 * SOLID or outside a non-periodic box, in x-fastest cell order, then alpha.
 * links: host int32 [count][4] = (x, y, z, alpha), or NULL to get the count
 * only.  *count receives the number of links.  EINVAL for bad sizes or flags. */
int lbm_wall_links(const uint8_t* mask, int nx, int ny, int nz, unsigned periodic_bits,
                   int32_t* links, int64_t* count);

/* Device bytes the caller must provide to lbm_attach_device. */
int lbm_device_bytes(const lbm_domain* dom, size_t* bytes);

/* Attach caller-owned device memory (at least lbm_device_bytes, 256-byte
 * aligned) and upload the node tables (asynchronous on the stream).  The
 * memory must outlive the domain.  ENOMEM if too small, EINVAL if misaligned. */
int lbm_attach_device(lbm_domain* dom, void* dev_ptr, size_t bytes);

/* Number of fluid nodes. */
int lbm_fluid_count(const lbm_domain* dom, int64_t* n);

/* Coordinates of the fluid nodes in library order: host int32 [n][3] = (x, y, z). */
int lbm_fluid_coords(const lbm_domain* dom, int32_t* xyz);

/* Set tau, the free rates and the body force (Eq. (6), Sec. 2.1.3).
 * EINVAL unless tau > 1/2, every s in (0, 2), all values finite. */
int lbm_set_params(lbm_domain* dom, const lbm_params* p);

/* Collision operator of a domain.  LBM_COLLISION_CHM_MRT (the default) is the
 * central Hermite MRT collision with the full equilibrium (Eq. (6)-(8)).
 * LBM_COLLISION_SRT2 is the classical comparator of Sec. 2.1.1-2.1.2: BGK
 * relaxation (Eq. (2)) with rate 1/tau towards the equilibrium of Eq. (3) cut
 * after its second-order term, w rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u),
 * with Guo's force populations (1 - 1/(2 tau)) w rho [3 (c - u).g
 * + 9 (c.u)(c.g)] and the same u = (j + rho g / 2) / rho; the free rates of
 * lbm_params are not used.  lbm_init_equilibrium then starts from that
 * operator's own equilibrium.  May be called at any time; the next step uses
 * it.  EINVAL for an unknown kind. */
enum { LBM_COLLISION_CHM_MRT = 0, LBM_COLLISION_SRT2 = 1 };
int lbm_set_collision(lbm_domain* dom, int kind);

/* Streaming pattern of lbm_step.  The step is the pull scheme of Sec. 2.1
 * (stream f_a(x, t+1) = f*_a(x - c_a, t), halfway bounce-back and the
 * open-boundary rules on the links whose source is not fluid) followed by the
 * collision; the pattern only decides where the populations are kept between
 * steps, never their values.
 * LBM_STREAM_PULL: two population buffers, each step reads one and writes the
 * other.
 * LBM_STREAM_INPLACE: one buffer, steps alternating between two kinds.  The
 * first reads f*_a(x - c_a, t) from slot abar of the source node (or the
 * node's own f*_abar from its slot a on a wall or open link) and writes
 * f*_abar(x, t+1) back to that same place; the next reads slot a of x and
 * writes f*_a(x, t+2) to slot abar of x.  Every place is read and written by
 * one node, so the buffer is updated in place; results are bitwise equal to
 * LBM_STREAM_PULL.  One buffer of populations fits the 256 MB Infinity Cache
 * where two may not, and every other step touches only its own node.
 * Readers of the state (lbm_moments, lbm_average, lbm_read_populations,
 * lbm_get_state) and batches first move the populations back to the pull
 * layout (one extra pass, on the domain's stream); the next in-place step
 * moves them again.  With curved walls (lbm_create_domain_curved) the
 * q >= 1/2 rule needs the node's own f*_a(x), whose slot another node
 * rewrites in place; the domain keeps it per wall link (one population per
 * weight record, part of lbm_device_bytes).  May be called at any time.
 * EINVAL for an unknown mode.
 * LBM_STREAM_AUTO (the default): in place for 4- and 8-byte populations
 * where the two buffers of the pull scheme exceed 192 MiB (they no longer
 * stay in the 256 MB Infinity Cache) and one buffer is at most 320 MiB; pull
 * otherwise.  Measured on the synthetic aneurysm at 256^3-512^3: in place
 * steps FP32 1.15-1.23 times faster at 105-218 MiB per buffer and FP64 1.16
 * and 1.07 times at 209 and 293 MiB; FP64 at 437 MiB and the 2-byte forms
 * (whose step is bound by vector instructions more than by memory) step
 * faster with pull, and so do curved walls (512^3 FP32: 100.3 us per step
 * with pull, 109.5 us in place), which LBM_STREAM_AUTO therefore never
 * streams in place. */
enum { LBM_STREAM_PULL = 0, LBM_STREAM_INPLACE = 1, LBM_STREAM_AUTO = 2 };
int lbm_set_streaming(lbm_domain* dom, int mode);

/* *in_place = 1 when lbm_step streams in place (the mode of
 * lbm_set_streaming resolved for this domain), else 0.  EINVAL for NULL. */
int lbm_streaming_in_place(const lbm_domain* dom, int* in_place);

/* Velocity inlet on the INLET ghost cells: the wall velocity of a link is
 * u_w = axis * U(r, t) at the link midpoint, where r is the distance from the
 * line through `center` along `axis` and U is the Womersley profile
 * U = G0 (R^2 - r^2) / (4 nu) + Re{ G1 / (i omega) [1 - J0(i^{3/2} a r / R)
 * / J0(i^{3/2} a)] e^{i omega t} }, a = R sqrt(omega / nu), U = 0 for r >= R,
 * and omega = 0 gives the steady Poiseuille profile.  The incoming population
 * is f_a(x, t+1) = f*_abar(x, t) + f_eq_a(1, u_w) - f_eq_abar(1, u_w)
 * (moving-wall bounce-back) with t the time of the populations being
 * streamed.  axis must be non-zero, radius > 0, values finite. */
int lbm_set_inlet_womersley(lbm_domain* dom, const double axis[3], const double center[3],
                            double radius, double G0, double G1, double omega);

/* Pressure outlet on the OUTLET ghost cells (default rho_out = 1, zero gauge
 * pressure): f_a(x, t+1) = -f*_abar(x, t) + f_eq_a(rho_out, u(x, t))
 * + f_eq_abar(rho_out, u(x, t)) (anti-bounce-back), with u(x, t) the
 * velocity of the node's last collision.  EINVAL unless rho_out > 0. */
int lbm_set_outlet_pressure(lbm_domain* dom, double rho_out);

/* Initial state at t = 0: f(0) = f_eq(rho, u) (product form of Eq. (3)),
 * followed by the first collision.  rho (device double [n]) and u (device
 * double [3][n]) may be NULL for rest (rho = 1, u = 0).  Needs attach and
 * params (ESTATE otherwise). */
int lbm_init_equilibrium(lbm_domain* dom, const double* rho, const double* u);

/* Advance nsteps >= 0 time steps (asynchronous).  Each step pulls
 * f(x, t+1) from the post-collision populations of step t, applies the
 * boundary rules, computes rho and u, collides (Eq. (6)) and stores the
 * post-collision populations; the same kernel writes per-block FP64 monitor
 * partials.  ESTATE before lbm_init_equilibrium. */
int lbm_step(lbm_domain* dom, int nsteps);

/* Current time index t (number of steps since initialisation). */
int lbm_time(const lbm_domain* dom, int64_t* t);

/* rho(t) (device double [n]) and u(t) (device double [3][n], component-major)
 * of the current state, in fluid-node order (Eqs. (4)-(5) with the half-force
 * velocity shift).  Either pointer may be NULL.  Asynchronous. */
int lbm_moments(lbm_domain* dom, double* rho, double* u);

/* Time averaging of u (FP64 accumulator in the attached memory).
 * op = LBM_AVG_RESET clears it (and stops tracking), LBM_AVG_ACCUMULATE adds
 * u(t) of the current state (a separate pass, u in FP64 from the stored
 * populations), LBM_AVG_TRACK makes every following step add the velocity it
 * computes for its collision (FP32 for the FP32/FP16/BF16 storage types, FP64
 * for FP64; no extra launch or pass) until RESET or lbm_init_equilibrium,
 * LBM_AVG_READ writes the mean of everything added since RESET to u_avg
 * (device double [3][n]; ESTATE if nothing was added).  Tracking also applies
 * to steps taken through a batch.  Asynchronous. */
enum { LBM_AVG_RESET = 0, LBM_AVG_ACCUMULATE = 1, LBM_AVG_READ = 2, LBM_AVG_TRACK = 3 };
int lbm_average(lbm_domain* dom, int op, double* u_avg);

/* Monitoring points (Sec. 2.2.2: the velocity at fixed points over several
 * cycles shows when the flow has become periodic).  nprobe <= 64 fluid cells
 * (x, y, z) = xyz[3k .. 3k+2] (host).  From the next step on, every step that
 * forms a time t with t - t_set a positive multiple of `every` writes record
 * r = (t - t_set) / every - 1 of the caller's device buffer
 * out_dev double [capacity][nprobe][4] = (rho, ux, uy, uz) of each probe at
 * time t: the values lbm_moments would report then, computed in the step
 * kernel's arithmetic precision.  t_set is the time of the call (0 again
 * after lbm_init_equilibrium).  Records beyond capacity are dropped.  out_dev
 * must stay valid while probes are set; nprobe = 0 removes them.  Errors:
 * EINVAL for a probe outside the box or not at a fluid cell, nprobe above 64,
 * every or capacity below 1, NULL or misaligned buffers; ESTATE without
 * device memory. */
int lbm_set_probes(lbm_domain* dom, const int32_t* xyz, int nprobe, int every, double* out_dev,
                   int64_t capacity);

/* Records written so far (at most the capacity). */
int lbm_probe_count(const lbm_domain* dom, int64_t* nrec);

/* Monitors of the last step (host double[10]); synchronizes the stream.
 * out = { mass sum rho, momentum sum j (3), wall force (3), inlet mass flux,
 * outlet mass flux, t }.  The wall force is the momentum the walls receive,
 * sum over wall links of 2 f*_abar c_abar; a flux is the mass a boundary
 * added in that step, so M(t) - M(t-1) = inlet + outlet flux.  Sums are FP64
 * in a fixed order (deterministic).  EUNSTABLE if any value is not finite;
 * ESTATE before the first step. */
int lbm_monitors(lbm_domain* dom, double out[10]);

/* Post-collision shifted populations f*(t) - w as FP64 (device double
 * [27][n], direction-major, alpha = 9 (cz+1) + 3 (cy+1) + (cx+1)).  Exact
 * conversion from the storage type.  Asynchronous. */
int lbm_read_populations(lbm_domain* dom, double* f_dev);

/* Checkpoint: raw state (populations in storage format and in the library's
 * pull layout, the open-boundary terms, time; a domain streamed in place is
 * brought back to that layout first).  With host == NULL, *bytes
 * receives the size; otherwise *bytes must be at least that size.
 * Synchronizes the stream. */
int lbm_get_state(lbm_domain* dom, void* host, size_t* bytes);

/* Restore a checkpoint taken from a domain with the same mask, storage and
 * row-tile edge.  EINVAL if the header does not match (including a state
 * written in another layout version).  Synchronizes the stream. */
int lbm_set_state(lbm_domain* dom, const void* host, size_t bytes);

/* Host-side evaluation of the inlet speed U(r, t) used by the velocity inlet
 * (same profile as lbm_set_inlet_womersley, with viscosity nu).  Pure host
 * computation; usable without a GPU.  EINVAL for radius <= 0, nu <= 0 or
 * non-finite r, t. */
int lbm_inlet_profile(double r, double t, double radius, double nu, double G0, double G1,
                      double omega, double* speed);

/* Free the host side of the domain (the caller frees the device memory). */
void lbm_destroy(lbm_domain* dom);

/* ---- Batched stepping -----------------------------------------------------
 * Many domains (uneven geometries, different tau) advanced by launches that
 * cover all of them, so small domains fill the device together.  The domains
 * keep their own memory, parameters and state; a batch step performs exactly
 * the per-node arithmetic of lbm_step, so every domain ends bit-identical to
 * stepping it alone.  All domains need the same storage type.  Batch work runs
 * on the batch's stream: the caller orders it against the domains' streams
 * (lbm_batch_step synchronizes each domain's stream before it enqueues). */

/* Create a batch of n >= 1 distinct attached domains (the pointer array is
 * copied; the domains must outlive the batch).  hip_stream: hipStream_t of
 * the batch work (must not be the NULL stream for graph capture). */
int lbm_batch_create(lbm_domain* const* doms, int n, void* hip_stream, lbm_batch** out);
int lbm_batch_device_bytes(const lbm_batch* batch, size_t* bytes);
/* Attach caller-owned device memory for the batch tables (256-byte aligned). */
int lbm_batch_attach_device(lbm_batch* batch, void* dev_ptr, size_t bytes);

/* Execution choice: cfg = { mode (0: one launch per step over the domains of
 * a group; 1: persistent launch looping over the group's work with a
 * device-wide barrier between steps; 2: one launch per step, every domain
 * streamed in place in one buffer, as lbm_set_streaming(LBM_STREAM_INPLACE)
 * steps it; needs work-group size 256 and no streaming stores, and
 * lbm_batch_step fails with EINVAL while a domain has curved-wall links),
 * work-group size (128, 256 or 512), streaming stores (0/1; 4- and 8-byte
 * storage only), persistent grid (0 = every work-group that fits at once),
 * group budget in MiB (0: all domains form one group; otherwise the domains
 * are split into as many groups of consecutive domains as the total
 * population working set (two buffers per domain, one in mode 2) divided by
 * the budget, rounded up, with near-equal working sets, and each group runs
 * all requested steps before the next, which keeps it in the device cache) }.
 * EINVAL for other values.  Mode 2 leaves the domains in an in-place layout:
 * readers of the state and lbm_step restore what they need first. */
int lbm_batch_config(const lbm_batch* batch, int cfg[5]);
int lbm_batch_set_config(lbm_batch* batch, const int cfg[5]);

/* Autotuner: time every configuration on this batch for about trial_steps
 * steps each (the domains advance by those steps; mode 2 only without curved
 * walls) and keep the fastest;
 * results are cached per process by storage, collision form, batch size
 * class and domain count.  best_ms_per_step (nullable) receives the best
 * time per step; when it is non-NULL the trials run even on a cache hit. */
int lbm_batch_autotune(lbm_batch* batch, int trial_steps, double* best_ms_per_step);

/* Advance every domain by nsteps (asynchronous on the batch stream; replays
 * captured graphs of 16 steps).  The last step writes every domain's
 * monitors (read them with lbm_monitors).  ESTATE unless every domain is
 * initialised. */
int lbm_batch_step(lbm_batch* batch, int nsteps);

/* Synchronize the batch stream; EDEVICE if a persistent launch hit the bound
 * of a device-wide barrier wait (its results are then invalid). */
int lbm_batch_status(lbm_batch* batch);

/* Free the host side of the batch (not the domains). */
void lbm_batch_destroy(lbm_batch* batch);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
