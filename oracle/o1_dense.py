"""Oracle tier O1: the CHM-MRT lattice Boltzmann step by its dense definitions.

TEST INFRASTRUCTURE ONLY -- see the package docstring.  Plain numpy, FP64,
dense box, array-of-structures populations ``f[z, y, x, alpha]``.

What one step computes (the evolution equation, Eq. (1), split as collide then
push-stream):

1. Conserved moments, Eqs. (4)-(5): rho = sum f, rho u = sum c f, with the
   half-force velocity shift u = (j + rho g / 2) / rho when a body force g acts.
2. Equilibrium by the Hermite series of Eq. (3) with the full expansion
   supported by D3Q27 (Sec. 2.1.3: sixth order), written out over tensor
   Hermite polynomials of every order 0..6.
3. CHM-MRT collision, Eq. (6): f* = f + T^-1 S T (f_eq - f) + T^-1 (I - S/2) F,
   with T the 27x27 central Hermite moment transform about the local u
   (Eqs. (7)-(8)), S diagonal with the six second-order rates equal to 1/tau
   and the orders 3..6 set by free rates (Sec. 2.1.3), and F the force's
   central Hermite moments (rho g in the three first-order rows).
4. Push streaming with halfway bounce-back at walls (Eq. (9) at q = 1/2),
   moving-wall bounce-back at velocity-inlet ghost cells and anti-bounce-back
   at pressure-outlet ghost cells (the bounce-back family of Sec. 2.1.2 used
   for velocity and pressure boundaries).

Readings where the paper is silent (basis of T, forcing, boundary formulas,
inlet profile) are the ones listed for the project; each function states its
own.
"""

from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.special

# --- D3Q27 lattice -----------------------------------------------------------
# Direction index alpha = 9 (cz + 1) + 3 (cy + 1) + (cx + 1); opposite = 26 - alpha.
C = np.array([(cx, cy, cz) for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)],
             dtype=np.int64)
OPP = np.array([26 - a for a in range(27)])
CS2 = 1.0 / 3.0
_W1 = {0: 2.0 / 3.0, 1: 1.0 / 6.0, -1: 1.0 / 6.0}
W = np.array([_W1[cx] * _W1[cy] * _W1[cz] for cx, cy, cz in C])

# Central Hermite moment index m = 9 k + 3 j + i for the polynomial
# H_i(xi_x) H_j(xi_y) H_k(xi_z), i, j, k in {0, 1, 2}; its order is i + j + k.
MIDX = [(i, j, k) for k in range(3) for j in range(3) for i in range(3)]
ORDER = np.array([i + j + k for i, j, k in MIDX])


def _h1(n, xi):
    """One-dimensional Hermite polynomial of degree n <= 2 (weight variance cs^2)."""
    if n == 0:
        return np.ones_like(xi)
    if n == 1:
        return xi
    return xi * xi - CS2


# --- Eq. (3): equilibrium as a Hermite series ----------------------------------

def _tensor_hermite_table(nmax: int = 6) -> dict:
    """Tensor Hermite polynomials H_{a1..an}(c_alpha) for every index tuple of
    order n <= nmax, evaluated at the 27 lattice velocities.

    Recursive definition (Grad): H^(0) = 1, H^(1)_a = xi_a and
    H^(n+1)_{a1..an b} = xi_b H^(n)_{a1..an} - cs^2 sum_k delta_{b ak} H^(n-1)_{a1..^ak..an}.
    """
    xi = C.astype(np.float64)
    table = {(): np.ones(27)}
    for n in range(1, nmax + 1):
        for tup in itertools.product(range(3), repeat=n):
            head, b = tup[:-1], tup[-1]
            val = xi[:, b] * table[head]
            for k, ak in enumerate(head):
                if ak == b:
                    val = val - CS2 * table[head[:k] + head[k + 1:]]
            table[tup] = val
    return table


_HTAB = _tensor_hermite_table(6)


def _supported(tup) -> bool:
    # On D3Q27 a tensor component is represented by the lattice only when no
    # Cartesian index appears more than twice (c^3 = c for c in {-1, 0, 1}).
    return all(tup.count(a) <= 2 for a in range(3))


def equilibrium_series(rho: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Eq. (3) with N = 6: f_eq = w sum_n (1 / (n! cs^2n)) a_n^eq : H_n,
    a_n^eq = rho u^{(x) n}, summed over every supported tensor component.

    rho: [N], u: [N, 3] -> f_eq: [N, 27].
    """
    rho = np.asarray(rho, np.float64)
    u = np.asarray(u, np.float64)
    acc = np.zeros((rho.shape[0], 27))
    for tup, h in _HTAB.items():
        if not _supported(tup):
            continue
        n = len(tup)
        coef = np.ones(rho.shape[0])
        for a in tup:
            coef = coef * u[:, a]
        acc += (coef / (math.factorial(n) * CS2 ** n))[:, None] * h[None, :]
    return W[None, :] * rho[:, None] * acc


def equilibrium_product(rho: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Closed-form product of the same expansion: rho prod_d psi(c_d, u_d) with
    psi(0, v) = 2/3 - v^2 and psi(+-1, v) = (1/3 + v^2 +- v)/2.  Used only by
    pins; the oracle's steps use :func:`equilibrium_series`."""
    rho = np.asarray(rho, np.float64)
    u = np.asarray(u, np.float64)
    out = np.ones((rho.shape[0], 27)) * rho[:, None]
    for d in range(3):
        v = u[:, d][:, None]
        c = C[:, d][None, :]
        psi = np.where(c == 0, 2.0 / 3.0 - v * v, (1.0 / 3.0 + v * v + c * v) / 2.0)
        out = out * psi
    return out


# --- Eq. (6)-(8): central Hermite moment transform ------------------------------

def central_transform(u: np.ndarray) -> np.ndarray:
    """T(u)[n, m, alpha] = H_i(c_x - u_x) H_j(c_y - u_y) H_k(c_z - u_z), m = 9k+3j+i."""
    u = np.asarray(u, np.float64)
    xi = C[None, :, :].astype(np.float64) - u[:, None, :]          # [N, 27, 3]
    T = np.empty((u.shape[0], 27, 27))
    for m, (i, j, k) in enumerate(MIDX):
        T[:, m, :] = _h1(i, xi[:, :, 0]) * _h1(j, xi[:, :, 1]) * _h1(k, xi[:, :, 2])
    return T


def relaxation_rates(tau: float, rates) -> np.ndarray:
    """Diagonal of S: order 0 and 1 -> 1 (their value does not matter), order 2
    -> 1/tau (the six viscous moments, Sec. 2.1.3), orders 3..6 -> free rates.

    ``rates`` is (s3, s4, s5, s6) or, for test hooks, (s2, s3, s4, s5, s6).
    """
    rates = tuple(float(r) for r in rates)
    if len(rates) == 4:
        s_by_order = (1.0, 1.0, 1.0 / tau) + rates
    elif len(rates) == 5:
        s_by_order = (1.0, 1.0) + rates
    else:
        raise ValueError("rates must have 4 or 5 entries")
    return np.array([s_by_order[o] for o in ORDER])


def moments(f: np.ndarray, g) -> tuple:
    """Eqs. (4)-(5) on [N, 27]: rho, raw momentum j, and u = (j + rho g/2) / rho."""
    rho = f.sum(axis=1)
    j = f @ C.astype(np.float64)
    u = (j + 0.5 * rho[:, None] * np.asarray(g, np.float64)[None, :]) / rho[:, None]
    return rho, j, u


def collide(f: np.ndarray, tau: float, rates, g) -> tuple:
    """One CHM-MRT collision on [N, 27] populations.

    Returns (f_post, rho, j, u).  Eq. (6) with the forcing term added in the
    same moment space: f* = f + T^-1 [ S T (f_eq - f) + (I - S/2) F ], where
    F has the central Hermite moments of the force, rho g in the first-order
    rows and zero elsewhere.
    """
    rho, j, u = moments(f, g)
    feq = equilibrium_series(rho, u)
    T = central_transform(u)
    s = relaxation_rates(tau, rates)
    F = np.zeros((f.shape[0], 27))
    gv = np.asarray(g, np.float64)
    for d, m in enumerate((1, 3, 9)):          # (1,0,0), (0,1,0), (0,0,1)
        F[:, m] = rho * gv[d]
    rhs = s[None, :] * np.einsum("nma,na->nm", T, feq - f) + (1.0 - 0.5 * s)[None, :] * F
    f_post = f + np.linalg.solve(T, rhs[:, :, None])[:, :, 0]
    return f_post, rho, j, u


# --- SRT comparator (Sec. 2.1.1-2.1.2) ------------------------------------------

def equilibrium_second_order(rho: np.ndarray, u: np.ndarray) -> np.ndarray:
    """The classical EDF: Eq. (3) truncated after the second-order term,
    w [rho + rho c.u / cs^2 + rho ((c.u)^2 - cs^2 u.u) / (2 cs^4)]."""
    cu = u @ C.T.astype(np.float64)                      # [N, 27]
    uu = (u * u).sum(axis=1)[:, None]
    return W[None, :] * rho[:, None] * (1.0 + cu / CS2 + (cu * cu - CS2 * uu) / (2.0 * CS2 * CS2))


def guo_force(rho: np.ndarray, u: np.ndarray, g) -> np.ndarray:
    """Force populations of Guo et al. for a force density rho g:
    w [(c - u) / cs^2 + (c.u) c / cs^4] . rho g."""
    gv = np.asarray(g, np.float64)
    Cf = C.astype(np.float64)
    cu = u @ Cf.T
    cg = Cf @ gv                                         # [27]
    ug = u @ gv                                          # [N]
    return W[None, :] * rho[:, None] * ((cg[None, :] - ug[:, None]) / CS2 + cu * cg[None, :] / (CS2 * CS2))


def collide_srt2(f: np.ndarray, tau: float, g) -> tuple:
    """Single-relaxation-time collision (Eq. (2)) towards the second-order EDF,
    with Guo's force term: f* = f + (f_eq2 - f) / tau + (1 - 1/(2 tau)) F.
    u = (j + rho g / 2) / rho as for CHM-MRT, so a step adds rho g of momentum."""
    rho, j, u = moments(f, g)
    f_post = f + (equilibrium_second_order(rho, u) - f) / tau + (1.0 - 0.5 / tau) * guo_force(rho, u, g)
    return f_post, rho, j, u


# --- Inlet profile --------------------------------------------------------------

def womersley_speed(r: np.ndarray, t: float, radius: float, nu: float,
                    G0: float, G1: float, omega: float) -> np.ndarray:
    """Axial speed of the Womersley solution in a pipe of the given radius under
    the pressure gradient G0 + G1 cos(omega t) per unit density.  Zero for
    r >= radius; steady Poiseuille when omega == 0."""
    r = np.asarray(r, np.float64)
    u = G0 * (radius * radius - r * r) / (4.0 * nu)
    if omega != 0.0 and G1 != 0.0:
        alpha = radius * math.sqrt(omega / nu)
        z0 = (1j) ** 1.5 * alpha
        ratio = scipy.special.jv(0, z0 * r / radius) / scipy.special.jv(0, z0)
        u = u + np.real(G1 / (1j * omega) * (1.0 - ratio) * np.exp(1j * omega * t))
    return np.where(r < radius, u, 0.0)


def inlet_velocity(points: np.ndarray, t: float, inlet, nu: float) -> np.ndarray:
    """Inlet wall velocity at the given points [N, 3] (link midpoints)."""
    axis = np.asarray(inlet.axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    d = points - np.asarray(inlet.center, np.float64)[None, :]
    perp = d - (d @ axis)[:, None] * axis[None, :]
    r = np.sqrt((perp * perp).sum(axis=1))
    spd = womersley_speed(r, t, inlet.radius, nu, inlet.G0, inlet.G1, inlet.omega)
    return spd[:, None] * axis[None, :]


# --- The step -------------------------------------------------------------------

class O1State:
    """Dense oracle state.

    ``f``  [nz, ny, nx, 27]  pre-collision populations at time ``t`` (zero off fluid)
    ``t``  time index
    ``u_last`` [nz, ny, nx, 3] velocity of the last collision (the outlet rule
    needs u(x, t) of the node whose populations it reflects).
    """

    def __init__(self, case, f=None, g_time=None):
        self.case = case
        self.mask = case.mask
        nz, ny, nx = case.mask.shape
        self.fluid = np.argwhere(case.mask == 1)            # [N, 3] as (z, y, x)
        self.f = np.zeros((nz, ny, nx, 27))
        if f is None:
            self.f[self.fluid[:, 0], self.fluid[:, 1], self.fluid[:, 2]] = W[None, :]
        else:
            self.f[...] = f
        self.t = 0
        self.u_last = np.zeros((nz, ny, nx, 3))
        # g(t) = g0 + g1 cos(omega_g t) for the Womersley pin; plain g otherwise.
        self.g_time = g_time
        self.monitors = None

    def g_at(self, t):
        if self.g_time is None:
            return np.asarray(self.case.g, np.float64)
        g0, g1, om = self.g_time
        return np.asarray(g0, np.float64) + np.asarray(g1, np.float64) * math.cos(om * t)

    def rates(self):
        return self.case.rates


def moving_wall_value(src: np.ndarray, feq_a: np.ndarray, feq_b: np.ndarray) -> np.ndarray:
    """Velocity inlet, moving-wall bounce-back (reading C8): the population that
    returns to the node is the one that left it towards the wall, plus
    f_eq_abar(1, u_w) - f_eq_a(1, u_w); a the direction into the wall."""
    return src + feq_b - feq_a


def anti_bounce_back_value(src: np.ndarray, feq_a: np.ndarray, feq_b: np.ndarray) -> np.ndarray:
    """Pressure outlet, anti-bounce-back (reading C9): minus the population
    that left towards the outlet, plus f_eq_a + f_eq_abar at (rho_out, u(x))."""
    return -src + feq_b + feq_a


def wall_force_of_links(src: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Momentum handed to the wall per step by halfway bounce-back links that
    leave with post-collision populations src in direction c: each reverses,
    so the fluid loses 2 f* c (momentum exchange)."""
    return 2.0 * src.sum() * c


def stream(state: O1State, f_post_nodes: np.ndarray, u_nodes: np.ndarray) -> tuple:
    """Push streaming of post-collision populations with the boundary rules.

    Returns (new dense f, wall force, inlet flux, outlet flux).  For a fluid node
    x and direction a with target y = x + c_a (periodic wrap on periodic axes):

    * y fluid:  f_a(y, t+1) = f*_a(x, t);
    * y wall (solid or outside the box): f_abar(x, t+1) = f*_a(x, t);
    * y inlet ghost:  f_abar(x, t+1) = f*_a(x, t) + f_eq_abar(1, u_w) - f_eq_a(1, u_w)
      with u_w the inlet velocity at the link midpoint x + c_a/2 at time t;
    * y outlet ghost: f_abar(x, t+1) = -f*_a(x, t) + f_eq_abar(rho_out, u(x,t))
      + f_eq_a(rho_out, u(x,t)).
    """
    case = state.case
    mask = case.mask
    nz, ny, nx = mask.shape
    dims = np.array([nz, ny, nx])
    per = np.array([bool(case.periodic & 4), bool(case.periodic & 2), bool(case.periodic & 1)])
    fl = state.fluid
    new = np.zeros_like(state.f)
    fwall = np.zeros(3)
    q_in = 0.0
    q_out = 0.0
    nu = case.nu
    for a in range(27):
        cz, cy, cx = C[a, 2], C[a, 1], C[a, 0]
        tgt = fl + np.array([cz, cy, cx])[None, :]
        inside = np.ones(len(fl), bool)
        for ax in range(3):
            if per[ax]:
                tgt[:, ax] %= dims[ax]
            else:
                inside &= (tgt[:, ax] >= 0) & (tgt[:, ax] < dims[ax])
        kind = np.zeros(len(fl), np.int64)                      # 0 -> wall
        ti = tgt[inside]
        kind[inside] = mask[ti[:, 0], ti[:, 1], ti[:, 2]]
        src = f_post_nodes[:, a]
        b = OPP[a]
        # fluid targets
        sel = kind == 1
        new[tgt[sel, 0], tgt[sel, 1], tgt[sel, 2], a] = src[sel]
        # walls
        sel = kind == 0
        new[fl[sel, 0], fl[sel, 1], fl[sel, 2], b] = src[sel]
        fwall += wall_force_of_links(src[sel], C[a].astype(np.float64))
        # inlet ghosts
        sel = kind == 2
        if np.any(sel):
            if case.inlet is None:
                raise ValueError("mask has inlet cells but the case has no inlet")
            mid = fl[sel][:, ::-1].astype(np.float64) + 0.5 * C[a][None, :]
            uw = inlet_velocity(mid, state.t, case.inlet, nu)
            feq = equilibrium_series(np.ones(len(uw)), uw)
            val = moving_wall_value(src[sel], feq[:, a], feq[:, b])
            new[fl[sel, 0], fl[sel, 1], fl[sel, 2], b] = val
            q_in += float((val - src[sel]).sum())
        # outlet ghosts
        sel = kind == 3
        if np.any(sel):
            ux = u_nodes[sel]
            feq = equilibrium_series(np.full(len(ux), case.rho_out), ux)
            val = anti_bounce_back_value(src[sel], feq[:, a], feq[:, b])
            new[fl[sel, 0], fl[sel, 1], fl[sel, 2], b] = val
            q_out += float((val - src[sel]).sum())
    return new, fwall, q_in, q_out


def step(state: O1State) -> None:
    """Advance the dense state by one time step (collide, then push-stream)."""
    fl = state.fluid
    f_nodes = state.f[fl[:, 0], fl[:, 1], fl[:, 2]]
    if getattr(state.case, "collision", "chm_mrt") == "srt2":
        f_post, rho, j, u = collide_srt2(f_nodes, state.case.tau, state.g_at(state.t))
    else:
        f_post, rho, j, u = collide(f_nodes, state.case.tau, state.rates(), state.g_at(state.t))
    state.u_last[fl[:, 0], fl[:, 1], fl[:, 2]] = u
    new, fwall, q_in, q_out = stream(state, f_post, u)
    state.f = new
    state.t += 1
    f1 = new[fl[:, 0], fl[:, 1], fl[:, 2]]
    mass = float(f1.sum())
    mom = f1 @ C.astype(np.float64)
    state.monitors = np.array([mass, *mom.sum(axis=0), *fwall, q_in, q_out, float(state.t)])
    state.last_post = f_post


def run(case, steps: int, f0=None, g_time=None) -> O1State:
    st = O1State(case, f0, g_time)
    for _ in range(steps):
        step(st)
    return st


def macroscopic(state: O1State) -> tuple:
    """rho [N] and u [N, 3] of the current (pre-collision) state, fluid nodes in
    (z, y, x) lexicographic order, i.e. x fastest."""
    fl = state.fluid
    f_nodes = state.f[fl[:, 0], fl[:, 1], fl[:, 2]]
    rho, _, u = moments(f_nodes, state.g_at(state.t))
    return rho, u
