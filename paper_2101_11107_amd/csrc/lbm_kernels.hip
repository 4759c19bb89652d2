// HIP kernels of the D3Q27 CHM-MRT lattice Boltzmann step for gfx950 (MI355X).
//
// One fused pull-scheme kernel per time step (Eq. (1)): every work-item owns
// one fluid node, gathers the 27 incoming post-collision populations of the
// previous step from the structure-of-arrays buffer (halfway bounce-back for
// wall links, Eq. (9) at q = 1/2; inlet/outlet rules for open links), forms
// rho and j (Eqs. (4)-(5)), applies the central Hermite moment collision
// (Eq. (6) with the equilibrium moments of Eq. (8)) with three one-dimensional
// transforms per direction in registers, and stores the 27 post-collision
// populations.  All populations are stored shifted by their weights
// (f - w_alpha) and the collision works on deviations, so every intermediate
// value is small and reduced-precision storage keeps its relative accuracy.
//
// Addressing: the neighbour of node (x, y, z) in row (y', z') is located from
// a fluid bitmap of the box and a per-word prefix count (the number of fluid
// nodes before that bitmap word in x-fastest order): the index of cell
// (x', y', z') is prefix + popcount of the preceding bits.  Only 4 bytes per
// node (its packed coordinates) are streamed besides the populations; the
// bitmap words are shared by a whole wavefront and stay in cache.
#include "lbm_internal.h"

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
    __device__ static T ld(const double* p, uint32_t k) { return p[k]; }
    __device__ static void st(double* p, uint32_t k, T v) { p[k] = v; }
};
template <> struct Traits<float> {
    using T = float;
    __device__ static T ld(const float* p, uint32_t k) { return p[k]; }
    __device__ static void st(float* p, uint32_t k, T v) { p[k] = v; }
};
template <> struct Traits<_Float16> {
    using T = float;
    __device__ static T ld(const _Float16* p, uint32_t k) { return (float)p[k]; }
    __device__ static void st(_Float16* p, uint32_t k, T v) { p[k] = (_Float16)v; }   // RNE
};
template <> struct Traits<__bf16> {
    using T = float;
    __device__ static T ld(const __bf16* p, uint32_t k) { return (float)p[k]; }
    __device__ static void st(__bf16* p, uint32_t k, T v) { p[k] = (__bf16)v; }       // RNE
};

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

// --- central Hermite transforms (one line of three populations) ---------------------
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

// Collision of the shifted populations f (= f - w) in place; returns u.
// Deviation form: with dA = T(u) f_hat and (T w)_ijk = p_i(ux) p_j(uy) p_k(uz),
// p = (1, -u, u^2), the post-collision deviations are
//   order 0: d rho;  order 1: rho g / 2 + u;  order n >= 2: (1 - s_n) dA - s_n (T w),
// and f_hat* = T(u)^-1 of them.
template <class T>
__device__ __forceinline__ void collide(T (&f)[27], T drho, T jx, T jy, T jz,
                                        const T (&om)[5], const T (&sr)[5], const T (&g)[3],
                                        T& ux, T& uy, T& uz) {
    const T rho = T(1) + drho;
    const T inv = T(1) / rho;
    const T hr = T(0.5) * rho;
    ux = (jx + hr * g[0]) * inv;
    uy = (jy + hr * g[1]) * inv;
    uz = (jz + hr * g[2]) * inv;
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

template <class T>
__device__ __forceinline__ void sums(const T (&f)[27], T& drho, T& jx, T& jy, T& jz) {
    // rho - 1 and j of the shifted populations (sum w = 1, sum w c = 0).
    T s[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) s[q] = f[3 * q] + f[3 * q + 1] + f[3 * q + 2];
    T x = T(0);
#pragma unroll
    for (int q = 0; q < 9; ++q) x += f[3 * q + 2] - f[3 * q];
    const T zm = s[0] + s[1] + s[2], z0 = s[3] + s[4] + s[5], zp = s[6] + s[7] + s[8];
    const T ym = s[0] + s[3] + s[6], yp = s[2] + s[5] + s[8];
    drho = zm + z0 + zp;
    jx = x;
    jy = yp - ym;
    jz = zp - zm;
}

// --- gather of the incoming populations ---------------------------------------------
template <class S>
__device__ __forceinline__ void gather_fast(const S* __restrict__ fin, const StepArgs& a, int i,
                                            uint32_t w, typename Traits<S>::T (&f)[27],
                                            uint32_t& wallmask) {
    const int x = w & 1023, y = (w >> 10) & 1023, z = (w >> 20) & 1023;
    const int wl = x >> 5, sh = x & 31;
    const uint32_t low = (uint32_t)((2ull << sh) - 1ull);
    const uint32_t np = (uint32_t)a.npad;
    const int rowlen = a.ny + 2;
#pragma unroll
    for (int kz = 0; kz < 3; ++kz) {
#pragma unroll
        for (int ky = 0; ky < 3; ++ky) {
            int ys = y - (ky - 1), zs = z - (kz - 1);
            if (a.periodic & 2) ys = ys < 0 ? ys + a.ny : (ys >= a.ny ? ys - a.ny : ys);
            if (a.periodic & 4) zs = zs < 0 ? zs + a.nz : (zs >= a.nz ? zs - a.nz : zs);
            const uint32_t row = (uint32_t)((zs + 1) * rowlen + (ys + 1)) * (uint32_t)a.W + wl;
            const uint32_t w0 = a.bits[row], w1 = a.bits[row + 1];
            const uint32_t b3 = (uint32_t)(((((uint64_t)w1) << 32) | w0) >> sh) & 7u;
            int base;
            if (ky == 1 && kz == 1) base = i;
            else base = a.prefix[row] + __popc(w0 & low);
#pragma unroll
            for (int kx = 0; kx < 3; ++kx) {
                const int al = 9 * kz + 3 * ky + kx;
                const int k = 2 - kx;              // bit of the source cell x - cx
                const bool fl = (b3 >> k) & 1u;
                const int src = (k == 0) ? base - 1 : (k == 1 ? base : base + (int)((b3 >> 1) & 1u));
                const uint32_t addr = fl ? (uint32_t)al * np + (uint32_t)src
                                         : (uint32_t)(26 - al) * np + (uint32_t)i;
                f[al] = Traits<S>::ld(fin, addr);
                if (!fl) wallmask |= 1u << al;
            }
        }
    }
}

template <class S>
__device__ __forceinline__ void gather_special(const S* __restrict__ fin, const StepArgs& a, int i,
                                            int sidx, typename Traits<S>::T (&f)[27], double (&F)[3],
                                            double& qin, double& qout) {
    using T = typename Traits<S>::T;
    const SpecialNode* sp = a.spec + sidx;
    const uint32_t np = (uint32_t)a.npad;
    const int64_t t = a.tcount[a.tin];
    double cw = 1.0, sw = 0.0;
    bool have_trig = false;
#pragma unroll
    for (int al = 0; al < 27; ++al) {
        const int code = sp->src[al];
        if (code >= 0) {
            f[al] = Traits<S>::ld(fin, (uint32_t)al * np + (uint32_t)code);
            continue;
        }
        const T own_t = Traits<S>::ld(fin, (uint32_t)(26 - al) * np + (uint32_t)i);
        const double own = (double)own_t;
        if (code == SRC_WALL) {
            f[al] = own_t;
            const double v = 2.0 * (own + wgt(al));
            F[0] -= v * cxo(al);
            F[1] -= v * cyo(al);
            F[2] -= v * czo(al);
            continue;
        }
        const BcLink L = a.links[-2 - code];
        double val;
        if (L.type == LINK_INLET) {
            if (!have_trig) {
                sincos(a.omega * (double)t, &sw, &cw);
                have_trig = true;
            }
            const double spd = L.a0 + L.a1re * cw - L.a1im * sw;
            const double uw[3] = {a.axis[0] * spd, a.axis[1] * spd, a.axis[2] * spd};
            val = own + (feq1(al, 1.0, uw) - feq1(26 - al, 1.0, uw));
            const T vt = (T)val;
            f[al] = vt;
            qin += (double)vt - own;
        } else {
            const double ux[3] = {a.u_spec[3 * sidx], a.u_spec[3 * sidx + 1], a.u_spec[3 * sidx + 2]};
            val = -own + ((feq1(al, a.rho_out, ux) - wgt(al)) + (feq1(26 - al, a.rho_out, ux) - wgt(al)));
            const T vt = (T)val;
            f[al] = vt;
            qout += (double)vt - own;
        }
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Fixed-order block reduction of 9 monitor values into partials[lb].
__device__ __forceinline__ void block_monitor(double (&m)[9], double* __restrict__ out) {
    __shared__ double red[BLOCK / 64][9];
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
        for (int q = 0; q < BLOCK / 64; ++q) s += red[q][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

template <class T>
__device__ __forceinline__ void load_rates(const StepArgs& a, T (&om)[5], T (&sr)[5], T (&g)[3]) {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        sr[k] = (T)a.s[k];
        om[k] = (T)(1.0 - a.s[k]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) g[d] = (T)a.g[d];
}

// --- the step kernel ----------------------------------------------------------------
// FULL = true also accumulates the wall force (momentum given to the walls).
template <class S, bool FULL>
__global__ __launch_bounds__(BLOCK) void k_step(StepArgs a) {
    using T = typename Traits<S>::T;
    // XCD-aware order: hardware work-group b runs on XCD (b % 8); give each XCD
    // a contiguous range of the node list so neighbour rows share its L2.
    const int hb = blockIdx.x;
    const int lb = (hb & 7) * a.blocks_per_xcd + (hb >> 3);
    if (lb >= a.nblocks) return;
    const int i = lb * BLOCK + threadIdx.x;
    const S* __restrict__ fin = (const S*)a.fin;
    S* __restrict__ fout = (S*)a.fout;
    double mon[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (i < a.n) {
        T f[27];
        uint32_t wallmask = 0;
        double F[3] = {0.0, 0.0, 0.0}, qin = 0.0, qout = 0.0;
        const uint32_t w = a.node[i];
        int sidx = -1;
        if (!(w & SPECIAL_BIT)) {
            gather_fast<S>(fin, a, i, w, f, wallmask);
        } else {
            sidx = (int)(w & ~SPECIAL_BIT);
            gather_special<S>(fin, a, i, sidx, f, F, qin, qout);
        }
        T drho, jx, jy, jz;
        sums(f, drho, jx, jy, jz);
        if (FULL && wallmask) {
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
        mon[0] = (double)drho;
        mon[1] = (double)jx;
        mon[2] = (double)jy;
        mon[3] = (double)jz;
        mon[4] = F[0];
        mon[5] = F[1];
        mon[6] = F[2];
        mon[7] = qin;
        mon[8] = qout;
        T om[5], sr[5], g[3];
        load_rates(a, om, sr, g);
        T ux, uy, uz;
        collide(f, drho, jx, jy, jz, om, sr, g, ux, uy, uz);
        if (sidx >= 0) {
            a.u_spec[3 * sidx] = (double)ux;
            a.u_spec[3 * sidx + 1] = (double)uy;
            a.u_spec[3 * sidx + 2] = (double)uz;
        }
        const uint32_t np = (uint32_t)a.npad;
#pragma unroll
        for (int al = 0; al < 27; ++al) Traits<S>::st(fout, (uint32_t)al * np + (uint32_t)i, f[al]);
    }
    if (lb == 0 && threadIdx.x == 0) a.tcount[a.tin ^ 1] = a.tcount[a.tin] + 1;
    block_monitor(mon, a.partials + (size_t)lb * MON_WORDS);
}

// Initial state: f(0) = f_eq(rho, u), then the first collision; written to fout.
template <class S>
__global__ __launch_bounds__(BLOCK) void k_init(StepArgs a, const double* rho0, const double* u0) {
    using T = typename Traits<S>::T;
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i == 0) {
        a.tcount[a.tin] = 0;
        a.tcount[a.tin ^ 1] = 0;
    }
    if (i >= a.n) return;
    const double r = rho0 ? rho0[i] : 1.0;
    const double u[3] = {u0 ? u0[i] : 0.0, u0 ? u0[a.n + i] : 0.0, u0 ? u0[2 * a.n + i] : 0.0};
    T f[27];
#pragma unroll
    for (int al = 0; al < 27; ++al) f[al] = (T)(feq1(al, r, u) - wgt(al));
    T drho, jx, jy, jz;
    sums(f, drho, jx, jy, jz);
    T om[5], sr[5], g[3];
    load_rates(a, om, sr, g);
    T ux, uy, uz;
    collide(f, drho, jx, jy, jz, om, sr, g, ux, uy, uz);
    const uint32_t w = a.node[i];
    if (w & SPECIAL_BIT) {
        const int sidx = (int)(w & ~SPECIAL_BIT);
        a.u_spec[3 * sidx] = (double)ux;
        a.u_spec[3 * sidx + 1] = (double)uy;
        a.u_spec[3 * sidx + 2] = (double)uz;
    }
    S* fout = (S*)a.fout;
    const uint32_t np = (uint32_t)a.npad;
#pragma unroll
    for (int al = 0; al < 27; ++al) Traits<S>::st(fout, (uint32_t)al * np + (uint32_t)i, f[al]);
}

// rho and u of the current state from the post-collision populations, in FP64:
// rho = 1 + sum f_hat*, u = (sum c f_hat* - rho g / 2) / rho (the collision adds
// rho g to j and keeps rho).  mode 0: write rho/u; 1: avg += u; 2: out = avg / count.
template <class S>
__global__ __launch_bounds__(BLOCK) void k_moments(StepArgs a, double* rho, double* u, double* avg,
                                                  int mode, double count) {
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
    const S* fin = (const S*)a.fin;
    const uint32_t np = (uint32_t)a.npad;
    double d = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int al = 0; al < 27; ++al) {
        const double v = (double)Traits<S>::ld(fin, (uint32_t)al * np + (uint32_t)i);
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
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= a.n) return;
    const S* fin = (const S*)a.fin;
    const uint32_t np = (uint32_t)a.npad;
#pragma unroll
    for (int al = 0; al < 27; ++al)
        out[(size_t)al * a.n + i] = (double)Traits<S>::ld(fin, (uint32_t)al * np + (uint32_t)i);
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
hipError_t step_t(const StepArgs& a, bool full, hipStream_t st) {
    const dim3 grid(8 * a.blocks_per_xcd), block(BLOCK);
    if (full) hipLaunchKernelGGL((k_step<S, true>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_step<S, false>), grid, block, 0, st, a);
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

hipError_t launch_step(int storage, const StepArgs& a, bool full, hipStream_t stream) {
    LBM_DISPATCH(storage, step_t, a, full, stream);
}

namespace {
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
