// Device code of the D3Q27 CHM-MRT step shared by the single-domain kernels
// (lbm_step.hip) and the batched kernels (lbm_batch.hip).
//
// One fused pull-scheme update per fluid node (Eq. (1)): gather the 27
// incoming post-collision populations of the previous step from the
// population buffer (pop_index layout: 256-byte runs of one direction per
// tile of nodes; halfway bounce-back for wall links,
// Eq. (9) at q = 1/2; inlet/outlet rules for open links), form rho and j
// (Eqs. (4)-(5)),
// apply the central Hermite moment collision (Eq. (6) with the equilibrium
// central moments (rho, 0, ..., 0) of Eq. (8)) in registers with
// one-dimensional transforms along x, y and z, and store the 27
// post-collision populations.  Populations are stored shifted by their
// weights (f - w_alpha) and the collision works on deviations, so every
// intermediate value is small and reduced-precision storage keeps its
// relative accuracy.
//
// Addressing: a node's neighbours in row (y', z') are located through a row
// table that holds, per 32 cells, the fluid bitmap word and the number of
// fluid nodes before it in list order: the index of fluid cell (x', y', z') is
// that count plus the popcount of the preceding bits.  Besides the
// populations only one 4-byte descriptor per node is streamed; the row table
// is shared by a wavefront and stays in cache.  Loads use 32-bit byte offsets
// from a uniform base, so each population address costs one or two integer
// operations.
#pragma once

#include "lbm_internal.h"

#include <type_traits>

namespace lbm {
namespace {

// --- lattice ------------------------------------------------------------------
// alpha = 9 (cz + 1) + 3 (cy + 1) + (cx + 1); opposite = 26 - alpha.
__host__ __device__ constexpr int cxo(int a) { return a % 3 - 1; }
__host__ __device__ constexpr int cyo(int a) { return (a / 3) % 3 - 1; }
__host__ __device__ constexpr int czo(int a) { return a / 9 - 1; }
__host__ __device__ constexpr double w1d(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double wgt(int a) { return w1d(cxo(a)) * w1d(cyo(a)) * w1d(czo(a)); }

// --- storage traits -------------------------------------------------------------
template <class S> struct Traits;
template <> struct Traits<double> {
    using T = double;
    __device__ static T cvt(double v) { return v; }
    __device__ static double store(T v) { return v; }
};
template <> struct Traits<float> {
    using T = float;
    __device__ static T cvt(float v) { return v; }
    __device__ static float store(T v) { return v; }
};
template <> struct Traits<_Float16> {
    using T = float;
    __device__ static T cvt(_Float16 v) { return (float)v; }
    __device__ static _Float16 store(T v) { return (_Float16)v; }    // round to nearest even
};
template <> struct Traits<__bf16> {
    using T = float;
    __device__ static T cvt(__bf16 v) { return (float)v; }
    __device__ static __bf16 store(T v) { return (__bf16)v; }        // round to nearest even
};

// Fused multiply-add in the arithmetic type (one rounding).
__device__ __forceinline__ float fma_rn(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_rn(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Load / store of one population at a byte offset from a uniform base.
// Population and table pointers reach the step as kernel arguments or, for
// batched stepping, from an argument table in memory; the explicit global
// address space keeps the accesses global (not generic flat) in both cases.
#define LBM_GLOBAL __attribute__((address_space(1)))

template <class S>
__device__ __forceinline__ typename Traits<S>::T ldp(const LBM_GLOBAL char* __restrict__ base, uint32_t off) {
    return Traits<S>::cvt(*(const LBM_GLOBAL S*)(base + off));
}
template <class S, bool NT = false>
__device__ __forceinline__ void stp(LBM_GLOBAL char* __restrict__ base, uint32_t off, typename Traits<S>::T v) {
    if (NT) __builtin_nontemporal_store(Traits<S>::store(v), (LBM_GLOBAL S*)(base + off));   // streaming store
    else *(LBM_GLOBAL S*)(base + off) = Traits<S>::store(v);
}

// Byte offsets of the population layout (pop_index: tiles of T nodes with
// their 27 directions as runs of T values) split into a part shared by the
// directions and a part shared by the nodes: population a of node n sits at
// node_off(n) + dir_off(a).  The direction part is uniform, so the kernels
// add it to the buffer's base (scalar arithmetic) and keep one per-lane
// offset for every direction.
template <class S>
__device__ __forceinline__ uint32_t node_off(uint32_t n) {
    constexpr uint32_t SZ = sizeof(S);
    return pop_index(n, 0u, 0u, SZ) * SZ;
}
__device__ __forceinline__ constexpr uint32_t dir_off(int al) { return (uint32_t)al * POP_RUN_BYTES; }

// Full-expansion equilibrium (product form of Eq. (3)) in FP64, one direction.
__device__ inline double feq1(int a, double rho, const double u[3]) {
    double r = rho;
    const int c[3] = {cxo(a), cyo(a), czo(a)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double v = u[d];
        r *= (c[d] == 0) ? (2.0 / 3.0 - v * v) : 0.5 * (1.0 / 3.0 + v * v + c[d] * v);
    }
    return r;
}

// Second-order equilibrium (Eq. (3) cut after n = 2) in FP64, one direction.
__device__ inline double feq2(int a, double rho, const double u[3]) {
    const double cu = cxo(a) * u[0] + cyo(a) * u[1] + czo(a) * u[2];
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    return wgt(a) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
}

// --- central Hermite transforms on one line (c = -1, 0, +1) ---------------------
// Forward: (f-, f0, f+) -> (m0, m1, m2) with H0 = 1, H1 = c - u, H2 = (c - u)^2 - 1/3.
template <class T>
__device__ __forceinline__ void fwd1(T& a, T& b, T& c, T u, T u2m) {
    const T m0 = a + b + c;
    const T d = c - a;
    const T s = c + a;
    a = m0;
    b = d - u * m0;
    c = s - T(2) * u * d + u2m * m0;          // u2m = u^2 - 1/3
}
// Inverse of fwd1.
template <class T>
__device__ __forceinline__ void inv1(T& a, T& b, T& c, T u, T u2p) {
    const T r1 = b + u * a;
    const T r2 = c + T(2) * u * b + u2p * a;  // u2p = u^2 + 1/3
    const T m0 = a;
    a = T(0.5) * (r2 - r1);
    b = m0 - r2;
    c = T(0.5) * (r2 + r1);
}
// Inverse with the first- and second-order inputs given at half scale
// (b = m1/2, c = m2/2): k = r1/2, h = r2/2, f- = h - k, f0 = m0 - 2h, f+ = h + k.
template <class T>
__device__ __forceinline__ void inv1h(T& a, T& b, T& c, T uh, T u2, T u2ph) {
    const T k = b + uh * a;                   // uh = u/2
    const T h = c + u2 * b + u2ph * a;        // u2 = 2u, u2ph = (u^2 + 1/3)/2
    const T m0 = a;
    a = h - k;
    b = m0 - T(2) * h;
    c = h + k;
}

// Line sums over x for the nine (cy, cz) lines q = 3 (cz + 1) + (cy + 1).
template <class T>
__device__ __forceinline__ void line_sums(const T (&f)[27], T (&S0)[9], T (&S1)[9], T (&S2)[9]) {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        S1[q] = f[3 * q + 2] - f[3 * q];
        S2[q] = f[3 * q + 2] + f[3 * q];
        S0[q] = S2[q] + f[3 * q + 1];
    }
}

template <class T>
__device__ __forceinline__ void conserved(const T (&S0)[9], const T (&S1)[9], T& drho, T& jx, T& jy, T& jz) {
    // rho - 1 and j of the shifted populations (sum w = 1, sum w c = 0)
    const T zm = S0[0] + S0[1] + S0[2], z0 = S0[3] + S0[4] + S0[5], zp = S0[6] + S0[7] + S0[8];
    const T ym = S0[0] + S0[3] + S0[6], yp = S0[2] + S0[5] + S0[8];
    drho = (zm + z0) + zp;
    jx = ((S1[0] + S1[1]) + (S1[2] + S1[3])) + ((S1[4] + S1[5]) + (S1[6] + S1[7])) + S1[8];
    jy = yp - ym;
    jz = zp - zm;
}

// General collision (any free rates), deviation form.  With dA = T(u) f_hat and
// (T w)_ijk = p_i(ux) p_j(uy) p_k(uz), p = (1, -u, u^2), the post-collision
// deviations are: order 0: d rho; order 1: rho g / 2 + u; order n >= 2:
// (1 - s_n) dA - s_n (T w); then f_hat* = T(u)^-1 of them.
template <class T>
__device__ __forceinline__ void collide_general(T (&f)[27], T drho, T ux, T uy, T uz, T hr,
                                                const T (&om)[5], const T (&sr)[5], const T (&g)[3]) {
    const T third = T(1) / T(3);
    const T xm = ux * ux - third, ym = uy * uy - third, zm = uz * uz - third;
#pragma unroll
    for (int q = 0; q < 9; ++q) fwd1(f[3 * q], f[3 * q + 1], f[3 * q + 2], ux, xm);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) fwd1(f[9 * k + i], f[9 * k + i + 3], f[9 * k + i + 6], uy, ym);
#pragma unroll
    for (int q = 0; q < 9; ++q) fwd1(f[q], f[q + 9], f[q + 18], uz, zm);

    const T px[3] = {T(1), -ux, ux * ux};
    const T py[3] = {T(1), -uy, uy * uy};
    const T pz[3] = {T(1), -uz, uz * uz};
#pragma unroll
    for (int m = 0; m < 27; ++m) {
        const int i = m % 3, j = (m / 3) % 3, k = m / 9, n = i + j + k;
        if (n == 0) {
            f[m] = drho;
        } else if (n == 1) {
            f[m] = (i == 1) ? hr * g[0] + ux : ((j == 1) ? hr * g[1] + uy : hr * g[2] + uz);
        } else {
            const T tw = px[i] * py[j] * pz[k];
            f[m] = om[n - 2] * f[m] - sr[n - 2] * tw;
        }
    }

    const T xp = ux * ux + third, yp = uy * uy + third, zp = uz * uz + third;
#pragma unroll
    for (int q = 0; q < 9; ++q) inv1(f[q], f[q + 9], f[q + 18], uz, zp);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) inv1(f[9 * k + i], f[9 * k + i + 3], f[9 * k + i + 6], uy, yp);
#pragma unroll
    for (int q = 0; q < 9; ++q) inv1(f[3 * q], f[3 * q + 1], f[3 * q + 2], ux, xp);
}

// Collision when the free rates of orders 3..6 all equal 1: those moments
// relax fully to equilibrium, so only the six second-order central moments of
// the incoming populations are needed.  They follow from the raw second
// moments P of f_hat:  dA_ab = P_ab - u_a j_b - u_b j_a + u_a u_b d rho
// - delta_ab d rho / 3.  Post-collision deviations: order 0 d rho, order 1
// rho g / 2 + u, order 2 (1 - s2) dA - s2 (T w), orders 3..6 -(T w).  The
// inverse runs with every moment scaled by 1/2 per non-zero index (inv1h).
template <class T>
__device__ __forceinline__ void collide_rates_one(T (&f)[27], const T (&S0)[9], const T (&S1)[9],
                                                  const T (&S2)[9], T drho, T jx, T jy, T jz,
                                                  T ux, T uy, T uz, T hr, T om2, T s2,
                                                  const T (&g)[3]) {
    const T third = T(1) / T(3);
    const T Pxx = ((S2[0] + S2[1]) + (S2[2] + S2[3])) + ((S2[4] + S2[5]) + (S2[6] + S2[7])) + S2[8];
    const T Pxy = (S1[2] + S1[5] + S1[8]) - (S1[0] + S1[3] + S1[6]);
    const T Pxz = (S1[6] + S1[7] + S1[8]) - (S1[0] + S1[1] + S1[2]);
    const T Pyy = (S0[0] + S0[2]) + (S0[3] + S0[5]) + (S0[6] + S0[8]);
    const T Pzz = (S0[0] + S0[1]) + (S0[2] + S0[6]) + (S0[7] + S0[8]);
    const T Pyz = (S0[0] + S0[8]) - (S0[2] + S0[6]);
    const T d3 = drho * third;
    const T dxx = Pxx - T(2) * ux * jx + (ux * ux) * drho - d3;
    const T dyy = Pyy - T(2) * uy * jy + (uy * uy) * drho - d3;
    const T dzz = Pzz - T(2) * uz * jz + (uz * uz) * drho - d3;
    const T dxy = Pxy - ux * jy - uy * jx + (ux * uy) * drho;
    const T dxz = Pxz - ux * jz - uz * jx + (ux * uz) * drho;
    const T dyz = Pyz - uy * jz - uz * jy + (uy * uz) * drho;

    // half-scaled p: q = (1, -u/2, u^2/2)
    const T qx[3] = {T(1), T(-0.5) * ux, T(0.5) * ux * ux};
    const T qy[3] = {T(1), T(-0.5) * uy, T(0.5) * uy * uy};
    const T qz[3] = {T(1), T(-0.5) * uz, T(0.5) * uz * uz};
    const T hom2 = T(0.5) * om2, qom2 = T(0.25) * om2;
    T m[27];
    m[0] = drho;
    m[1] = T(0.5) * (hr * g[0] + ux);
    m[3] = T(0.5) * (hr * g[1] + uy);
    m[9] = T(0.5) * (hr * g[2] + uz);
    // order 2, scaled by 1/2 (one non-zero index) or 1/4 (two)
    m[2] = hom2 * dxx - s2 * qx[2];
    m[6] = hom2 * dyy - s2 * qy[2];
    m[18] = hom2 * dzz - s2 * qz[2];
    m[4] = qom2 * dxy - s2 * (qx[1] * qy[1]);
    m[10] = qom2 * dxz - s2 * (qx[1] * qz[1]);
    m[12] = qom2 * dyz - s2 * (qy[1] * qz[1]);
    // orders 3..6 with 1 - s = 0: -(T w), scaled
#pragma unroll
    for (int mm = 0; mm < 27; ++mm) {
        const int i = mm % 3, j = (mm / 3) % 3, k = mm / 9;
        if (i + j + k >= 3) m[mm] = -(qx[i] * qy[j]) * qz[k];
    }
    const T uhz = T(0.5) * uz, u2z = T(2) * uz, u2pz = T(0.5) * (uz * uz + third);
    const T uhy = T(0.5) * uy, u2y = T(2) * uy, u2py = T(0.5) * (uy * uy + third);
    const T uhx = T(0.5) * ux, u2x = T(2) * ux, u2px = T(0.5) * (ux * ux + third);
    // z pass; the lines (i, j) with i + j >= 3 hold -(T w) only and invert to
    // -(q_i q_j) w1(cz)
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int i = q % 3, j = q / 3;
        if (i + j >= 3) {
            const T P = qx[i] * qy[j];
            const T e = P * T(-1.0 / 6.0);
            m[q] = e;
            m[q + 9] = P * T(-2.0 / 3.0);
            m[q + 18] = e;
        } else {
            inv1h(m[q], m[q + 9], m[q + 18], uhz, u2z, u2pz);
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) inv1h(m[9 * k + i], m[9 * k + i + 3], m[9 * k + i + 6], uhy, u2y, u2py);
#pragma unroll
    for (int q = 0; q < 9; ++q) inv1h(m[3 * q], m[3 * q + 1], m[3 * q + 2], uhx, u2x, u2px);
#pragma unroll
    for (int mm = 0; mm < 27; ++mm) f[mm] = m[mm];
}

// --- gather of the incoming populations -------------------------------------------
// Row-table entry of a source row at the node's x (one 8-byte load).
typedef uint32_t RowWord2 __attribute__((ext_vector_type(2)));

// Ordinary node: streaming and halfway bounce-back through the row table.
// The nine row-table entries are loaded first and the population loads issued
// after all of them (vector loads retire in order, so interleaving them would
// serialize the rows).
// MODE STREAM_PULL: the pull layout.  MODE STREAM_NEIGHBOUR: the reversed
// layout of in-place streaming: direction al comes from slot abar of the
// source node, or from slot al of this node on a wall link; loc[al] keeps
// that byte offset (from fin), where f*_abar of this node is written back.
// MODE GATHER_WALL_BITS: no population loads, only the wall links.
constexpr int GATHER_WALL_BITS = 3;
template <class S, bool PER, bool WALLS, int MODE = STREAM_PULL>
__device__ __forceinline__ void gather_fast(const LBM_GLOBAL char* __restrict__ fin, const StepArgs& a, int i,
                                            uint32_t w, typename Traits<S>::T (&f)[27],
                                            uint32_t& wallmask, uint32_t (&loc)[27]) {
    constexpr uint32_t SZ = sizeof(S);
    const LBM_GLOBAL char* rt = (const LBM_GLOBAL char*)a.rowtab;
    const int x = (int)(w & 1023u);
    int y = 0, z = 0;
    uint32_t e0 = 0;
    const uint32_t kw = ((uint32_t)x * 2185u) >> 16;   // x / ROW_SPAN (exact for x < 1024)
    if (!PER) {
        e0 = (w >> 10) * (uint32_t)a.W + kw;
    } else {
        y = (int)((w >> 10) & 1023u);
        z = (int)((w >> 20) & 1023u);
    }
    const uint32_t sh = (uint32_t)x - (uint32_t)ROW_SPAN * kw;   // bit of cell x - 1
    const uint32_t low = (2u << sh) - 1u;                         // cells 30k - 1 .. x - 1
    const int rowlen = a.ny + 2;
    RowWord2 rp[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int ky = q % 3, kz = q / 3;
        uint32_t e;
        if (!PER) {
            e = e0 - (uint32_t)(((ky - 1) + (kz - 1) * rowlen) * a.W);
        } else {
            int ys = y - (ky - 1), zs = z - (kz - 1);
            if (a.periodic & 2) ys = ys < 0 ? ys + a.ny : (ys >= a.ny ? ys - a.ny : ys);
            if (a.periodic & 4) zs = zs < 0 ? zs + a.nz : (zs >= a.nz ? zs - a.nz : zs);
            e = (uint32_t)((zs + 1) * rowlen + (ys + 1)) * (uint32_t)a.W + kw;
        }
        rp[q] = *(const LBM_GLOBAL RowWord2*)(rt + e * 8u);
    }
    __builtin_amdgcn_sched_barrier(0);
    const uint32_t own = node_off<S>((uint32_t)i);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int ky = q % 3, kz = q / 3;
        // bits of cells x - 1, x, x + 1 of this row
        const uint32_t win = rp[q].x >> sh;
        const int base = (q == 4) ? i : (int)rp[q].y + (int)__popc(rp[q].x & low);
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
            const int al = 9 * kz + 3 * ky + kx;
            const int k = 2 - kx;              // bit of the source cell x - cx
            if (al == 13) {
                if (MODE == STREAM_NEIGHBOUR) loc[13] = own + dir_off(13);
                if (MODE != GATHER_WALL_BITS) f[al] = ldp<S>(fin + dir_off(13), own);
                continue;
            }
            const bool fl = (win >> k) & 1u;
            if (MODE == GATHER_WALL_BITS) {
                if (!fl) wallmask |= 1u << al;
                continue;
            }
            const int src = (k == 0) ? base - 1 : (k == 1 ? base : base + (int)((win >> 1) & 1u));
            if (MODE == STREAM_NEIGHBOUR) {
                loc[al] = fl ? node_off<S>((uint32_t)src) + dir_off(26 - al) : own + dir_off(al);
                f[al] = ldp<S>(fin, loc[al]);
                if (WALLS && !fl) wallmask |= 1u << al;
                continue;
            }
            // pulled value: direction al of the source node; bounce-back:
            // direction abar of this node.  Both offsets are taken from the
            // lower of the two directions' runs, so that neither is negative.
            const int lo = al < 13 ? al : 26 - al;
            const uint32_t gap = dir_off(26 - 2 * lo);     // run(hi) - run(lo)
            const uint32_t pull = node_off<S>((uint32_t)src) + (al > 13 ? gap : 0u);
            const uint32_t bounce = own + (al < 13 ? gap : 0u);
            f[al] = ldp<S>(fin + dir_off(lo), fl ? pull : bounce);
            if (WALLS && !fl) wallmask |= 1u << al;
        }
    }
}

// Node with open-boundary or periodic-x links: explicit byte offsets, then the
// open-boundary corrections with the additive terms prepared by the previous
// step (or the initial state): inlet f_a = f*_abar + add, outlet
// f_a = -f*_abar + add (evaluated in FP64, rounded once).  wall_force: add the
// halfway wall force of the wall links to F (the curved-wall blend adds it
// otherwise).
// In-place streaming (IP = STREAM_NEIGHBOUR, STREAM_LOCAL) reads the same
// values from the places the layout gives them (see STREAM_PULL); own is
// node_off of this node, and loc receives the neighbour step's offsets.  The
// node-local step's values (the node's own slots) are loaded by the caller.
template <class S>
__device__ __forceinline__ uint32_t inplace_special_off(const LBM_GLOBAL SpecialNode* __restrict__ sp, int al,
                                                        uint32_t nonfluid, uint32_t own) {
    // a fluid source (also across a periodic x edge): slot abar instead of
    // slot al of that node; a wall or open link: slot al of this node
    return ((nonfluid >> al) & 1u) ? own + dir_off(al) : sp->off[al] - dir_off(al) + dir_off(26 - al);
}

template <class S, bool MON, int IP = STREAM_PULL>
__device__ __forceinline__ void gather_special(const LBM_GLOBAL char* __restrict__ fin, const StepArgs& a,
                                               const LBM_GLOBAL SpecialNode* __restrict__ sp,
                                               typename Traits<S>::T (&f)[27], double (&F)[3],
                                               double& qin, double& qout, bool wall_force,
                                               uint32_t (&loc)[27], uint32_t own) {
    using T = typename Traits<S>::T;
    const uint32_t wm = sp->wallmask, lm = sp->linkmask;
#pragma unroll
    for (int al = 0; al < 27; ++al) {
        if (IP == STREAM_PULL) {
            f[al] = ldp<S>(fin, sp->off[al]);
        } else if (IP == STREAM_NEIGHBOUR) {
            loc[al] = inplace_special_off<S>(sp, al, wm | lm, own);
            f[al] = ldp<S>(fin, loc[al]);
        }
        // STREAM_LOCAL: the caller has loaded the node's own slots into f
    }
    if (MON && wall_force && wm) {
#pragma unroll
        for (int al = 0; al < 27; ++al) {
            if ((wm >> al) & 1u) {
                const double v = 2.0 * ((double)f[al] + wgt(al));
                F[0] -= v * cxo(al);
                F[1] -= v * cyo(al);
                F[2] -= v * czo(al);
            }
        }
    }
    if (lm) {
        int l = sp->link0;
        const LBM_GLOBAL int32_t* meta = (const LBM_GLOBAL int32_t*)a.link_meta;
        const LBM_GLOBAL double* add = (const LBM_GLOBAL double*)a.link_add;
#pragma unroll
        for (int al = 0; al < 27; ++al) {
            if ((lm >> al) & 1u) {
                const bool inlet = (meta[l] & 0xff) == LINK_INLET;
                const double own = (double)f[al];
                const T vt = (T)((inlet ? own : -own) + add[l]);
                f[al] = vt;
                if (MON) {
                    const double q = (double)vt - own;
                    if (inlet) qin += q;
                    else qout += q;
                }
                ++l;
            }
        }
    }
}

// Curved walls (Eq. (9)-(10)), after the gather: each wall link's
// bounce-back value f[al] = f*_abar(x) becomes
// w0 f*_abar(x) + (1 - w0) f2, with the weight record r of the link (the
// layout is described at CREC_CHUNK): f2 = f[abar] = f*_abar(x + c_al), the
// value pulled for direction abar, for r > 0 (q < 1/2), and the node's own
// f*_al(x) for r < 0 (q >= 1/2).  A link whose q < 1/2 rule lacks its second
// node has r = 1, so f[abar] is never read where it is itself a wall value.
// The records of one direction of a wavefront are consecutive, so a lane finds
// its record from the wavefront's ballot of that direction; directions without
// a wall link in the wavefront are skipped.  The directions are taken in two
// halves, each issuing its record and second-value loads together; the first
// half's loads go out with the gather's.  With MON, the
// wall force of each link, (f*_abar(x) + f_al(x, t+1)) c_abar in full
// populations, is subtracted from F.  Streamed in place (IP != STREAM_PULL)
// the node's own f*_al(x) sits in a slot another node rewrites during the
// step, so it comes from the record's entry of a.cside instead, which
// curved_side_store refreshes after the collision.
template <class S, bool MON, int IP = STREAM_PULL>
__device__ __forceinline__ void curved_blend(const LBM_GLOBAL char* __restrict__ fin, const StepArgs& a, int i,
                                             uint32_t own0, uint32_t wallmask, typename Traits<S>::T (&f)[27],
                                             double (&F)[3]) {
    // rounding pinned (one fused multiply-add per blend, no other fusion), so
    // that every kernel built from this body rounds alike
#pragma clang fp contract(off)
    using T = typename Traits<S>::T;
    constexpr uint32_t SZ = sizeof(S);
    const LBM_GLOBAL T* __restrict__ rec = (const LBM_GLOBAL T*)a.crec;
    // the chunk of 64 nodes is the wavefront's (blocks are whole wavefronts)
    const int chunk = __builtin_amdgcn_readfirstlane(i / CREC_CHUNK);
    uint32_t cum = ((const LBM_GLOBAL uint32_t*)a.crec_base)[chunk];
    T fx = T(0), fy = T(0), fz = T(0);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        // a lane without the link keeps r = 1, f2 = 0: its blend returns
        // f[al] unchanged, so the blend needs no per-lane test
        T r[13], f2[13];
        unsigned long long B[13];
#pragma unroll
        for (int k = 0; k < 13; ++k) {
            const int al = 14 * h + k;
            const bool wl = (wallmask >> al) & 1u;
            B[k] = __ballot(wl);
            r[k] = T(1);
            f2[k] = T(0);
            if (B[k] != 0ull) {
                const uint32_t idx = __builtin_amdgcn_mbcnt_hi((uint32_t)(B[k] >> 32),
                                                               __builtin_amdgcn_mbcnt_lo((uint32_t)B[k], cum));
                cum += (uint32_t)__popcll(B[k]);
                if (wl) {
                    r[k] = rec[idx];
                    if (IP == STREAM_PULL) f2[k] = ldp<S>(fin + dir_off(al), own0);
                    else f2[k] = Traits<S>::cvt(((const LBM_GLOBAL S*)a.cside)[idx]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 13; ++k) {
            const int al = 14 * h + k;
            if (B[k] == 0ull) continue;
            const T own = f[al];
            const bool hi = r[k] < T(0);
            const T w0 = hi ? -r[k] : r[k];
            const T v = fma_rn(w0, own, (T(1) - w0) * (hi ? f2[k] : f[26 - al]));
            f[al] = v;
            if (MON) {
                // this lane's bit of the ballot (not of wallmask: reusing that
                // test would keep one register per direction alive across the loads)
                const T on = (T)(uint32_t)((B[k] >> __lane_id()) & 1ull);
                const T m = on * (own + v + T(2) * (T)wgt(al));
                if (cxo(al)) fx += cxo(al) > 0 ? m : -m;
                if (cyo(al)) fy += cyo(al) > 0 ? m : -m;
                if (czo(al)) fz += czo(al) > 0 ? m : -m;
            }
        }
        if (h == 0) {
            // the second half's loads stay behind the first half's blend, so
            // the two halves never hold their loaded values at once
#pragma unroll
            for (int k = 0; k < 13; ++k) asm volatile("" : "+v"(f[k]) : : "memory");
        }
    }
    if (MON) {
        F[0] -= (double)fx;
        F[1] -= (double)fy;
        F[2] -= (double)fz;
    }
}

// Curved walls streamed in place: after the collision, each wall link's record
// entry of a.cside takes the node's post-collision f*_al(x) (in the storage
// type, rounded as the population store rounds it), for the next step's
// blend.  Records in the blend's order: per 64-node chunk, then direction
// (al = 0..26 without 13), then node.
template <class S>
__device__ __forceinline__ void curved_side_store(const StepArgs& a, int i, uint32_t wallmask,
                                                  const typename Traits<S>::T (&f)[27]) {
    LBM_GLOBAL S* side = (LBM_GLOBAL S*)a.cside;
    const int chunk = __builtin_amdgcn_readfirstlane(i / CREC_CHUNK);
    uint32_t cum = ((const LBM_GLOBAL uint32_t*)a.crec_base)[chunk];
#pragma unroll
    for (int al = 0; al < 27; ++al) {
        if (al == 13) continue;
        const bool wl = (wallmask >> al) & 1u;
        const unsigned long long B = __ballot(wl);
        if (B == 0ull) continue;
        const uint32_t idx = __builtin_amdgcn_mbcnt_hi((uint32_t)(B >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)B, cum));
        cum += (uint32_t)__popcll(B);
        if (wl) side[idx] = Traits<S>::store(f[al]);
    }
}

// Additive terms of a special node's open links for the step that streams the
// populations of time t_next.  The inlet phase (cos, sin)(omega t_next) is read
// from the device phase slots.
__device__ __forceinline__ void update_links(const StepArgs& a, const LBM_GLOBAL SpecialNode* __restrict__ sp,
                                          double ux, double uy, double uz, int64_t t_next) {
    const int l0 = sp->link0, nl = __popc(sp->linkmask);
    const LBM_GLOBAL double* trig = (const LBM_GLOBAL double*)a.trig;
    const double cw = trig[2 * (t_next & 1)], sw = trig[2 * (t_next & 1) + 1];
    LBM_GLOBAL double* link_add = (LBM_GLOBAL double*)a.link_add;
    for (int l = l0; l < l0 + nl; ++l) {
        const int meta = ((const LBM_GLOBAL int32_t*)a.link_meta)[l];
        const int al = meta >> 8;
        const LBM_GLOBAL double* cf = (const LBM_GLOBAL double*)a.link_coef + LINK_COEFS * l;
        double add;
        if ((meta & 0xff) == LINK_INLET) {
            const double U = cf[0] + cf[1] * cw - cf[2] * sw;
            const double U2 = U * U;
            add = U * (cf[3] + U2 * (cf[4] + U2 * cf[5]));
        } else {
            // f_eq_a + f_eq_abar = 2 rho_out (even part of prod_d (e_d + o_d)),
            // e_d, o_d the even and odd parts of psi(c_d, u_d)
            const int c[3] = {al % 3 - 1, (al / 3) % 3 - 1, al / 9 - 1};
            const double u[3] = {ux, uy, uz};
            double e[3], o[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double v = u[d];
                e[d] = c[d] == 0 ? 2.0 / 3.0 - v * v : 0.5 * (1.0 / 3.0 + v * v);
                o[d] = c[d] == 0 ? 0.0 : 0.5 * c[d] * v;
            }
            const double even = e[0] * e[1] * e[2] + e[0] * o[1] * o[2] + o[0] * e[1] * o[2] + o[0] * o[1] * e[2];
            const double w = (c[0] == 0 ? 2.0 / 3.0 : 1.0 / 6.0) * (c[1] == 0 ? 2.0 / 3.0 : 1.0 / 6.0) *
                             (c[2] == 0 ? 2.0 / 3.0 : 1.0 / 6.0);
            add = 2.0 * (a.rho_out * even - w);
        }
        link_add[l] = add;
    }
}

// Advance the inlet phase: slot (t + 2) & 1 <- rotation of slot (t + 1) & 1 by
// omega, renormalized to unit length.
__device__ __forceinline__ void advance_phase(const StepArgs& a, int64_t t) {
    const double* p = a.trig + 2 * ((t + 1) & 1);
    const double c = p[0] * a.cos_w - p[1] * a.sin_w;
    const double s = p[1] * a.cos_w + p[0] * a.sin_w;
    const double r = 1.0 / sqrt(c * c + s * s);
    double* q = a.trig + 2 * ((t + 2) & 1);
    q[0] = c * r;
    q[1] = s * r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Fixed-order block reduction of 9 monitor values into out[0..8].
template <int BS>
__device__ __forceinline__ void block_monitor(double (&m)[9], double* __restrict__ out) {
    __shared__ double red[BS / 64][9];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = wave_sum(m[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 9; ++k) red[wv][k] = m[k];
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < BS / 64; ++q) s += red[q][threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();   // red may be reused by the block's next work item
}

// SRT comparator (Sec. 2.1.1-2.1.2): BGK relaxation (Eq. (2)) of the shifted
// populations towards the equilibrium of Eq. (3) cut after its second-order
// term, f_eq2 - w = w (drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)), plus Guo's
// force populations (1 - om/2) w rho [3 (c - u).g + 9 (c.u)(c.g)], om = 1/tau.
template <class T>
__device__ __forceinline__ void collide_srt2(T (&f)[27], T drho, T ux, T uy, T uz, T om, const T (&g)[3],
                                             bool force) {
    const T rho = T(1) + drho;
    const T uu = ux * ux + uy * uy + uz * uz;
    const T ug = ux * g[0] + uy * g[1] + uz * g[2];
    const T fo = (T(1) - T(0.5) * om) * rho;
#pragma unroll
    for (int al = 0; al < 27; ++al) {
        const int cx = cxo(al), cy = cyo(al), cz = czo(al);
        const T cu = (cx ? (cx > 0 ? ux : -ux) : T(0)) + (cy ? (cy > 0 ? uy : -uy) : T(0)) +
                     (cz ? (cz > 0 ? uz : -uz) : T(0));
        const T w = (T)wgt(al);
        const T feq = w * (drho + rho * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu));
        T v = f[al] - om * (f[al] - feq);
        if (force) {
            const T cg = (cx ? (cx > 0 ? g[0] : -g[0]) : T(0)) + (cy ? (cy > 0 ? g[1] : -g[1]) : T(0)) +
                         (cz ? (cz > 0 ? g[2] : -g[2]) : T(0));
            v += fo * w * (T(3) * (cg - ug) + T(9) * cu * cg);
        }
        f[al] = v;
    }
}

// Collision of the gathered populations (in place): moments, then one of the
// collision forms (FORM 0: CHM-MRT with general rates, 1: CHM-MRT with the
// free rates one, 2: the SRT comparator).  Returns the velocity and the
// conserved sums.
template <class T, int FORM>
__device__ __forceinline__ void collide(T (&f)[27], const StepArgs& a, T& ux, T& uy, T& uz, T& drho,
                                        T& jx, T& jy, T& jz) {
    T S0[9], S1[9], S2[9];
    line_sums(f, S0, S1, S2);
    conserved(S0, S1, drho, jx, jy, jz);
    T g[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) g[d] = (T)a.g[d];
    const T rho = T(1) + drho;
    const T inv = T(1) / rho;
    const T hr = T(0.5) * rho;
    ux = (jx + hr * g[0]) * inv;
    uy = (jy + hr * g[1]) * inv;
    uz = (jz + hr * g[2]) * inv;
    if (FORM == 1) {
        collide_rates_one(f, S0, S1, S2, drho, jx, jy, jz, ux, uy, uz, hr, (T)(1.0 - a.s[0]), (T)a.s[0], g);
    } else if (FORM == 2) {
        collide_srt2(f, drho, ux, uy, uz, (T)a.s[0], g, a.g[0] != 0.0 || a.g[1] != 0.0 || a.g[2] != 0.0);
    } else {
        T om[5], sr[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            sr[k] = (T)a.s[k];
            om[k] = (T)(1.0 - a.s[k]);
        }
        collide_general(f, drho, ux, uy, uz, hr, om, sr, g);
    }
}

// --- one block of a step ---------------------------------------------------------
// Logical block lb of the domain (BS consecutive nodes).  Used by the
// single-domain kernel and by the batched kernels, so a node's arithmetic is
// the same in both.  CURVED: blend the curved-wall links of ordinary nodes
// (a domain without weight records skips it).  IP: the streaming pattern
// (STREAM_PULL between fin and fout; the in-place steps with fin == fout read
// and write the places described at STREAM_PULL, with the same values and
// arithmetic as the pull step).
template <class S, bool MON, int FORM, bool PER, bool NT, int BS, bool CURVED, int IP = STREAM_PULL>
__device__ __forceinline__ void step_block(const StepArgs& a, int lb) {
    using T = typename Traits<S>::T;
    constexpr uint32_t SZ = sizeof(S);
    const int i = lb * BS + threadIdx.x;
    // the two buffers are distinct only for the pull step
    using InPtr = std::conditional_t<IP == STREAM_PULL, const LBM_GLOBAL char* __restrict__, const LBM_GLOBAL char*>;
    using OutPtr = std::conditional_t<IP == STREAM_PULL, LBM_GLOBAL char* __restrict__, LBM_GLOBAL char*>;
    const InPtr fin = (const LBM_GLOBAL char*)a.fin;
    const OutPtr fout = (LBM_GLOBAL char*)a.fout;
    double mon[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (i < a.n) {
        T f[27];
        uint32_t wallmask = 0;
        double F[3] = {0.0, 0.0, 0.0}, qin = 0.0, qout = 0.0;
        // the node's own population offset without its direction part (curved
        // walls, in-place streaming)
        const uint32_t own0 = (CURVED || IP != STREAM_PULL) ? node_off<S>((uint32_t)i) : 0u;
        if (IP == STREAM_LOCAL) {
            // every node of the node-local step reads its own slots: issued
            // before the descriptor says what kind of node this is
#pragma unroll
            for (int al = 0; al < 27; ++al) f[al] = ldp<S>(fin + dir_off(al), own0);
        }
        const LBM_GLOBAL SpecialNode* sp = nullptr;
        const bool curved = CURVED && a.crec != nullptr;
        uint32_t w;
        if (IP == STREAM_LOCAL && !MON) {
            // the node-local step needs a node's descriptor only for special
            // nodes (and curved walls): a wavefront without any skips it
            const uint32_t chunk = __builtin_amdgcn_readfirstlane((uint32_t)i / 64u);
            const bool any = ((const LBM_GLOBAL uint32_t*)a.wave_special)[chunk] != 0u;
            w = (any || curved) ? ((const LBM_GLOBAL uint32_t*)a.node)[i] : 0u;
        } else {
            w = ((const LBM_GLOBAL uint32_t*)a.node)[i];
        }
        // in-place neighbour step: where each direction was read
        uint32_t loc[27];
        if (!(w & SPECIAL_BIT)) {
            if (IP == STREAM_LOCAL) {
                if (MON || curved) gather_fast<S, PER, true, GATHER_WALL_BITS>(fin, a, i, w, f, wallmask, loc);
            } else {
                gather_fast<S, PER, MON || CURVED, IP>(fin, a, i, w, f, wallmask, loc);
            }
        } else {
            sp = (const LBM_GLOBAL SpecialNode*)a.spec + (w & ~SPECIAL_BIT);
            // read before the gather's loads, so that using it waits for none of them
            if (curved) wallmask = sp->wallmask;
            gather_special<S, MON, IP>(fin, a, sp, f, F, qin, qout, !curved, loc, own0);
        }
        if (curved) {
            // every wall link has a record (r = 1: halfway)
            if (__ballot(wallmask != 0u)) curved_blend<S, MON, IP>(fin, a, i, own0, wallmask, f, F);
        } else if (MON && wallmask) {
            T fx = T(0), fy = T(0), fz = T(0);
#pragma unroll
            for (int al = 0; al < 27; ++al) {
                if (al == 13) continue;
                const T v = ((wallmask >> al) & 1u) ? f[al] + (T)wgt(al) : T(0);
                if (cxo(al)) fx += cxo(al) > 0 ? v : -v;
                if (cyo(al)) fy += cyo(al) > 0 ? v : -v;
                if (czo(al)) fz += czo(al) > 0 ? v : -v;
            }
            F[0] -= 2.0 * (double)fx;
            F[1] -= 2.0 * (double)fy;
            F[2] -= 2.0 * (double)fz;
        }
        T ux, uy, uz, drho, jx, jy, jz;
        collide<T, FORM>(f, a, ux, uy, uz, drho, jx, jy, jz);
        if (a.nprobe > 0) {
            // monitoring points: the state this step forms is time tn
            const int64_t dt = a.tcount[a.tin] + 1 - a.probe_t0;
            if (dt > 0 && dt % a.probe_every == 0) {
                const int64_t rec = dt / a.probe_every - 1;
                if (rec < a.probe_cap) {
                    const LBM_GLOBAL int32_t* pn = (const LBM_GLOBAL int32_t*)a.probe_node;
                    for (int p = 0; p < a.nprobe; ++p) {
                        if (pn[p] == i) {
                            LBM_GLOBAL double* o = (LBM_GLOBAL double*)a.probe_out + (rec * a.nprobe + p) * 4;
                            o[0] = 1.0 + (double)drho;
                            o[1] = (double)ux;
                            o[2] = (double)uy;
                            o[3] = (double)uz;
                        }
                    }
                }
            }
        }
        if (a.avg != nullptr) {
            // running sum of the velocity of every step (each node its own entries)
            LBM_GLOBAL double* avg = (LBM_GLOBAL double*)a.avg;
            avg[i] += (double)ux;
            avg[a.n + i] += (double)uy;
            avg[2 * a.n + i] += (double)uz;
        }
        if (MON) {
            mon[0] = (double)drho;
            mon[1] = (double)jx;
            mon[2] = (double)jy;
            mon[3] = (double)jz;
            mon[4] = F[0];
            mon[5] = F[1];
            mon[6] = F[2];
            mon[7] = qin;
            mon[8] = qout;
        }
        if (IP != STREAM_PULL && curved) {
            if (__ballot(wallmask != 0u)) curved_side_store<S>(a, i, wallmask, f);
        }
        if (IP == STREAM_PULL) {
#pragma unroll
            for (int al = 0; al < 27; ++al) stp<S, NT>(fout + dir_off(al), node_off<S>((uint32_t)i), f[al]);
        } else if (IP == STREAM_NEIGHBOUR) {
            // f*_abar goes where direction al was read: the source node's slot
            // abar (the value it pulls next), or this node's slot al
#pragma unroll
            for (int al = 0; al < 27; ++al) stp<S, NT>(fout, loc[al], f[26 - al]);
        } else {
#pragma unroll
            for (int al = 0; al < 27; ++al) stp<S, NT>(fout + dir_off(26 - al), own0, f[al]);
        }
        // after the stores, so the populations are no longer live
        if (sp != nullptr && sp->linkmask != 0u)
            update_links(a, sp, (double)ux, (double)uy, (double)uz, a.tcount[a.tin] + 1);
    }
    if (lb == 0 && threadIdx.x == 0) {
        const int64_t t = a.tcount[a.tin];
        a.tcount[a.tin ^ 1] = t + 1;
        advance_phase(a, t);
    }
    if (MON) block_monitor<BS>(mon, a.partials + (size_t)lb * MON_WORDS);
}

}  // namespace
}  // namespace lbm
