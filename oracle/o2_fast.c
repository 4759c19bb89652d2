/*
 * Oracle tier O2: fast FP64 CPU implementation of the D3Q27 CHM-MRT step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link or call
 * this file; it exists to check the HIP library and to serve as the timed CPU
 * baseline.  It shares no code with the HIP library or with tier O1.
 *
 * Layout: fluid nodes in x-fastest order, array-of-structures f[n][27] in
 * FP64, plus a dense cell -> node index map.  One step = collide every node,
 * then push-stream (Eq. (1)).
 *
 * Collision (Eq. (6)-(8)): the central Hermite moments about the local u are
 * obtained by three one-dimensional transforms (x, then y, then z) of the
 * tensor-product basis H_i(c_x-u_x) H_j(c_y-u_y) H_k(c_z-u_z), H0 = 1,
 * H1 = xi, H2 = xi^2 - 1/3.  Because the full-expansion equilibrium has central
 * moments (rho, 0, ..., 0) (Eq. (8)), relaxation sets order 0 to rho, order 1
 * to rho g / 2 (force moment rho g applied with (1 - s/2)), and scales every
 * order n >= 2 moment by (1 - s_n); s_2 = 1/tau ties the six second-order
 * moments to the viscosity (Sec. 2.1.3).  The inverse transform runs z, y, x.
 *
 * Streaming: fluid -> fluid copy; halfway bounce-back at walls (Eq. (9) at
 * q = 1/2); moving-wall bounce-back at inlet ghosts with the Womersley
 * velocity at the link midpoint; anti-bounce-back at outlet ghosts with the
 * node's own velocity.
 *
 * Curved walls (Sec. 2.1.4, Eq. (9)-(10), the linear interpolation of Bouzidi
 * et al. that the paper cites): when a wall distance q (fraction of the link
 * from the node to the wall) is given for the link of node x in direction a
 * (x + c_a solid), the population returning to x in direction abar is
 *   q <  1/2: 2q f*_a(x) + (1 - 2q) f*_a(x - c_a)   (x - c_a must be fluid,
 *             otherwise the link keeps halfway bounce-back),
 *   q >= 1/2: f*_a(x) / (2q) + (2q - 1) / (2q) f*_abar(x),
 * both equal to halfway bounce-back at q = 1/2.  The wall force of such a link
 * is (f*_a(x) + f_abar(x, t + 1)) c_a (momentum exchange).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* Real type of the oracle's arithmetic.  double by default; built with
 * -DO2_LONG_DOUBLE every population, moment, equilibrium and sum is long
 * double (the x87 80-bit format with gcc on x86-64), which measures the
 * rounding floor of the double build.  Case parameters and the inlet profile
 * stay double: they are inputs. */
#ifdef O2_LONG_DOUBLE
typedef long double real;
#define RC(x) x##L
#else
typedef double real;
#define RC(x) x
#endif

typedef struct {
    int nx, ny, nz;
    unsigned periodic;          /* bit0 x, bit1 y, bit2 z */
    double tau;
    double s[5];                /* rates of orders 2..6 (s[0] normally 1/tau) */
    double g0[3], g1[3];        /* g(t) = g0 + g1 cos(omega_g t) */
    double omega_g;
    double rho_out;
    int has_inlet;
    double axis[3], center[3], radius, G0, G1, omega, nu;
    int collision;              /* 0 CHM-MRT, 1 SRT with the second-order EDF */
} o2_case;

static int CXYZ[27][3];
static real WGT[27];
static int OPPD[27];
static int tables_ready = 0;

static void init_tables(void) {
    if (tables_ready) return;
    const real w1[3] = {RC(1.0) / RC(6.0), RC(2.0) / RC(3.0), RC(1.0) / RC(6.0)};
    for (int cz = -1; cz <= 1; ++cz)
        for (int cy = -1; cy <= 1; ++cy)
            for (int cx = -1; cx <= 1; ++cx) {
                int a = 9 * (cz + 1) + 3 * (cy + 1) + (cx + 1);
                CXYZ[a][0] = cx; CXYZ[a][1] = cy; CXYZ[a][2] = cz;
                WGT[a] = w1[cx + 1] * w1[cy + 1] * w1[cz + 1];
                OPPD[a] = 26 - a;
            }
    tables_ready = 1;
}

/* Product-form full-expansion equilibrium for one direction. */
static real feq_dir(int a, real rho, const real u[3]) {
    real r = rho;
    for (int d = 0; d < 3; ++d) {
        real v = u[d];
        int c = CXYZ[a][d];
        r *= (c == 0) ? (RC(2.0) / RC(3.0) - v * v) : (RC(1.0) / RC(3.0) + v * v + c * v) * 0.5;
    }
    return r;
}

/* Complex Bessel J0 by its power series sum_k (-z^2/4)^k / (k!)^2. */
static double complex bessel_j0(double complex z) {
    double complex q = -z * z / 4.0, term = 1.0, sum = 1.0;
    for (int k = 1; k < 200; ++k) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (cabs(term) < 1e-18 * cabs(sum)) break;
    }
    return sum;
}

static double inlet_speed(const o2_case* c, double r, double t) {
    if (r >= c->radius) return 0.0;
    double u = c->G0 * (c->radius * c->radius - r * r) / (4.0 * c->nu);
    if (c->omega != 0.0 && c->G1 != 0.0) {
        double alpha = c->radius * sqrt(c->omega / c->nu);
        double complex i32 = cexp(I * 0.75 * M_PI);      /* i^(3/2) */
        double complex ratio = bessel_j0(i32 * alpha * r / c->radius) / bessel_j0(i32 * alpha);
        double complex amp = c->G1 / (I * c->omega) * (1.0 - ratio);
        u += creal(amp * cexp(I * c->omega * t));
    }
    return u;
}

/* 1-D forward transform of the triple (fm, f0, fp) at c = -1, 0, +1. */
static inline void fwd1(real* a, real* b, real* c, real u) {
    real fm = *a, f0 = *b, fp = *c;
    real m0 = fm + f0 + fp, d = fp - fm;
    *a = m0;
    *b = d - u * m0;
    *c = (fp + fm) - 2.0 * u * d + (u * u - RC(1.0) / RC(3.0)) * m0;
}

static inline void inv1(real* a, real* b, real* c, real u) {
    real m0 = *a, m1 = *b, m2 = *c;
    real r1 = m1 + u * m0;
    real r2 = m2 + 2.0 * u * m1 + (u * u + RC(1.0) / RC(3.0)) * m0;
    *a = 0.5 * (r2 - r1);
    *b = m0 - r2;
    *c = 0.5 * (r2 + r1);
}

static void collide_node(const o2_case* c, const real* f, real* fp, real* uo, const real g[3]) {
    real rho = 0, j[3] = {0, 0, 0};
    for (int a = 0; a < 27; ++a) {
        rho += f[a];
        for (int d = 0; d < 3; ++d) j[d] += CXYZ[a][d] * f[a];
    }
    real u[3];
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * rho * g[d]) / rho;
    real m[27];
    memcpy(m, f, sizeof m);
    for (int q = 0; q < 9; ++q) fwd1(&m[3 * q], &m[3 * q + 1], &m[3 * q + 2], u[0]);
    for (int kz = 0; kz < 3; ++kz)
        for (int i = 0; i < 3; ++i) {
            int b = 9 * kz + i;
            fwd1(&m[b], &m[b + 3], &m[b + 6], u[1]);
        }
    for (int q = 0; q < 9; ++q) fwd1(&m[q], &m[q + 9], &m[q + 18], u[2]);
    for (int k = 0; k < 3; ++k)
        for (int jj = 0; jj < 3; ++jj)
            for (int i = 0; i < 3; ++i) {
                int idx = 9 * k + 3 * jj + i, n = i + jj + k;
                if (n == 0) m[idx] = rho;
                else if (n == 1) m[idx] = 0.5 * rho * g[i == 1 ? 0 : (jj == 1 ? 1 : 2)];
                else m[idx] *= (RC(1.0) - (real)c->s[n - 2]);
            }
    for (int q = 0; q < 9; ++q) inv1(&m[q], &m[q + 9], &m[q + 18], u[2]);
    for (int kz = 0; kz < 3; ++kz)
        for (int i = 0; i < 3; ++i) {
            int b = 9 * kz + i;
            inv1(&m[b], &m[b + 3], &m[b + 6], u[1]);
        }
    for (int q = 0; q < 9; ++q) inv1(&m[3 * q], &m[3 * q + 1], &m[3 * q + 2], u[0]);
    memcpy(fp, m, sizeof m);
    for (int d = 0; d < 3; ++d) uo[d] = u[d];
}

/* SRT comparator (Sec. 2.1.1-2.1.2): BGK relaxation (Eq. (2)) towards the
 * equilibrium of Eq. (3) cut after its second-order term,
 *   feq2_a = w_a rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u),
 * plus Guo's force populations (1 - 1/(2 tau)) w_a rho [3 (c - u).g + 9 (c.u)(c.g)];
 * u = (j + rho g / 2) / rho as for CHM-MRT. */
static void collide_node_srt2(const o2_case* c, const real* f, real* fp, real* uo, const real g[3]) {
    real rho = 0, j[3] = {0, 0, 0};
    for (int a = 0; a < 27; ++a) {
        rho += f[a];
        for (int d = 0; d < 3; ++d) j[d] += CXYZ[a][d] * f[a];
    }
    real u[3];
    for (int d = 0; d < 3; ++d) u[d] = (j[d] + 0.5 * rho * g[d]) / rho;
    const real uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const real ug = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
    const real om = RC(1.0) / (real)c->tau;
    for (int a = 0; a < 27; ++a) {
        real cu = 0, cg = 0;
        for (int d = 0; d < 3; ++d) {
            cu += CXYZ[a][d] * u[d];
            cg += CXYZ[a][d] * g[d];
        }
        const real feq = WGT[a] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        const real F = WGT[a] * rho * (3.0 * (cg - ug) + 9.0 * cu * cg);
        fp[a] = f[a] - om * (f[a] - feq) + (1.0 - 0.5 * om) * F;
    }
    for (int d = 0; d < 3; ++d) uo[d] = u[d];
}

static void g_at(const o2_case* c, int64_t t, real g[3]) {
    real cs = cos(c->omega_g * (double)t);
    for (int d = 0; d < 3; ++d) g[d] = c->g0[d] + c->g1[d] * cs;
}

/* Collide every fluid node: f -> fpost, u. */
int o2_collide(const o2_case* c, int64_t n, const real* f, real* fpost, real* u,
               int64_t t, int nthreads) {
    init_tables();
    real g[3];
    g_at(c, t, g);
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (c->collision == 1) collide_node_srt2(c, f + 27 * i, fpost + 27 * i, u + 3 * i, g);
        else collide_node(c, f + 27 * i, fpost + 27 * i, u + 3 * i, g);
    }
    return 0;
}

/* Push-stream post-collision populations into fnew.
 * coords: [n][3] (x, y, z) of each node; idx: dense map cell -> node or -1.
 * mon_out[5]: wall force (3), inlet flux, outlet flux. */
int o2_stream(const o2_case* c, const uint8_t* mask, const int32_t* coords, const int32_t* idx,
              int64_t n, const real* fpost, const real* u, real* fnew, int64_t t,
              real* mon_out, int nthreads, const real* wq) {
    init_tables();
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const int dims[3] = {nx, ny, nz};
    const int per[3] = {(int)(c->periodic & 1), (int)((c->periodic >> 1) & 1), (int)((c->periodic >> 2) & 1)};
    real ax[3] = {c->axis[0], c->axis[1], c->axis[2]};
    real an = sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
    if (c->has_inlet) for (int d = 0; d < 3; ++d) ax[d] /= an;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    int nt = omp_get_max_threads();
    real* part = (real*)calloc((size_t)nt * 5, sizeof(real));
    int bad = 0;
#pragma omp parallel
    {
        real* pm = part + 5 * omp_get_thread_num();
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            const int* p = coords + 3 * i;
            for (int a = 0; a < 27; ++a) {
                int q[3], inside = 1;
                for (int d = 0; d < 3; ++d) {
                    q[d] = p[d] + CXYZ[a][d];
                    if (per[d]) q[d] = (q[d] + dims[d]) % dims[d];
                    else if (q[d] < 0 || q[d] >= dims[d]) inside = 0;
                }
                int kind = 0;
                size_t cell = 0;
                if (inside) {
                    cell = ((size_t)q[2] * ny + q[1]) * nx + q[0];
                    kind = mask[cell];
                }
                real src = fpost[27 * i + a];
                int b = OPPD[a];
                if (kind == 1) {
                    fnew[27 * (int64_t)idx[cell] + a] = src;
                } else if (kind == 2) {
                    real mid[3], dd[3], pr = 0, r2 = 0, uw[3];
                    for (int d = 0; d < 3; ++d) { mid[d] = p[d] + 0.5 * CXYZ[a][d]; dd[d] = mid[d] - c->center[d]; pr += dd[d] * ax[d]; }
                    for (int d = 0; d < 3; ++d) { real e = dd[d] - pr * ax[d]; r2 += e * e; }
                    real sp = c->has_inlet ? inlet_speed(c, sqrt(r2), (real)t) : 0.0;
                    if (!c->has_inlet) bad = 1;
                    for (int d = 0; d < 3; ++d) uw[d] = sp * ax[d];
                    real v = src + feq_dir(b, 1.0, uw) - feq_dir(a, 1.0, uw);
                    fnew[27 * i + b] = v;
                    pm[3] += v - src;
                } else if (kind == 3) {
                    const real* ux = u + 3 * i;
                    real v = -src + feq_dir(b, c->rho_out, ux) + feq_dir(a, c->rho_out, ux);
                    fnew[27 * i + b] = v;
                    pm[4] += v - src;
                } else {
                    real v = src;
                    const real q = wq ? wq[27 * i + a] : 0.5;
                    if (q >= 0.5) {
                        v = src / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * fpost[27 * i + b];
                    } else {
                        /* the node behind x along -c_a */
                        int r[3], ok = 1;
                        for (int d = 0; d < 3; ++d) {
                            r[d] = p[d] - CXYZ[a][d];
                            if (per[d]) r[d] = (r[d] + dims[d]) % dims[d];
                            else if (r[d] < 0 || r[d] >= dims[d]) ok = 0;
                        }
                        int64_t j = -1;
                        if (ok) {
                            size_t cr = ((size_t)r[2] * ny + r[1]) * nx + r[0];
                            if (mask[cr] == 1) j = idx[cr];
                        }
                        if (j >= 0) v = 2.0 * q * src + (1.0 - 2.0 * q) * fpost[27 * j + a];
                    }
                    fnew[27 * i + b] = v;
                    for (int d = 0; d < 3; ++d) pm[d] += (src + v) * CXYZ[a][d];
                }
            }
        }
    }
    for (int d = 0; d < 5; ++d) mon_out[d] = 0;
    for (int k = 0; k < nt; ++k)
        for (int d = 0; d < 5; ++d) mon_out[d] += part[5 * k + d];
    free(part);
    return bad ? -1 : 0;
}

/* Mass and momentum of a population array: out[4]. */
void o2_mass_momentum(int64_t n, const real* f, real* out) {
    init_tables();
    real m = 0, p[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 27; ++a) {
            real v = f[27 * i + a];
            m += v;
            for (int d = 0; d < 3; ++d) p[d] += CXYZ[a][d] * v;
        }
    out[0] = m; out[1] = p[0]; out[2] = p[1]; out[3] = p[2];
}

/* Run nsteps of collide + stream.  f (in/out) holds pre-collision populations
 * at time t0; fpost and u are work arrays that hold, on return, the last
 * post-collision populations and velocities.  mon[10] = mass, momentum (3),
 * wall force (3), inlet flux, outlet flux, time of the returned state. */
int o2_run(const o2_case* c, const uint8_t* mask, const int32_t* coords, const int32_t* idx,
           int64_t n, real* f, real* fpost, real* u, int64_t t0, int nsteps,
           real* mon, int nthreads, const real* wq) {
    int rc = 0;
    real m5[5] = {0, 0, 0, 0, 0};
    for (int s = 0; s < nsteps; ++s) {
        int64_t t = t0 + s;
        o2_collide(c, n, f, fpost, u, t, nthreads);
        rc |= o2_stream(c, mask, coords, idx, n, fpost, u, f, t, m5, nthreads, wq);
    }
    real mm[4];
    o2_mass_momentum(n, f, mm);
    mon[0] = mm[0]; mon[1] = mm[1]; mon[2] = mm[2]; mon[3] = mm[3];
    for (int d = 0; d < 5; ++d) mon[4 + d] = m5[d];
    mon[9] = (real)(t0 + nsteps);
    return rc;
}
