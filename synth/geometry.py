"""Seeded voxel geometries and case parameters.

Mask encoding (one byte per voxel, array index ``mask[z, y, x]``):

* ``SOLID``  (0) -- wall material; a link from a fluid node into it is a wall
  link (halfway bounce-back, Eq. (9) at q = 1/2);
* ``FLUID``  (1) -- a lattice node that is updated;
* ``INLET``  (2) -- ghost cell of a velocity inlet;
* ``OUTLET`` (3) -- ghost cell of a pressure outlet.

A node is fluid when the geometric predicate holds *strictly* at its integer
coordinate; ties are solid.  Out-of-box neighbours on a non-periodic axis are
walls.  Periodic axes are flagged by the ``PERIODIC_*`` bits.

The aneurysm family is a planar half-torus vessel (major radius 80, tube radius
12 at the 256^3 reference size) standing on two straight legs, with a spherical
sac fused at the outer bend.  It replaces the idealized sidewall aneurysm of the
paper (Sec. 2.2.2), whose CAD is not available; the Womersley number 3 used
for the inlet is close to the paper's 2.54 (Sec. 2.2.2).

Everything here is integer/geometry bookkeeping and scalar case parameters.
No lattice Boltzmann arithmetic lives in this module.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SOLID, FLUID, INLET, OUTLET = 0, 1, 2, 3
PERIODIC_X, PERIODIC_Y, PERIODIC_Z = 1, 2, 4


@dataclasses.dataclass
class Inlet:
    """Parameters of a Womersley velocity inlet (lattice units).

    The inlet velocity points along ``axis``; its magnitude depends on the
    distance r of a point from the line through ``center`` along ``axis``.
    ``G0`` and ``G1`` are the steady and oscillating pressure-gradient
    amplitudes (per unit density), ``omega`` the angular frequency; with
    ``omega == 0`` the profile is the steady Poiseuille one.  The kinematic
    viscosity the profile uses is the fluid's, ``(tau - 1/2) / 3``.
    """
    axis: tuple
    center: tuple
    radius: float
    G0: float
    G1: float
    omega: float


@dataclasses.dataclass
class Case:
    name: str
    mask: np.ndarray                 # uint8 [nz, ny, nx]
    periodic: int = 0
    tau: float = 0.8
    rates: tuple = (1.0, 1.0, 1.0, 1.0)   # free rates of orders 3, 4, 5, 6
    g: tuple = (0.0, 0.0, 0.0)           # body acceleration
    rho_out: float = 1.0
    inlet: Optional[Inlet] = None
    steps: int = 0
    period: int = 0
    seed: int = 0
    meta: dict = dataclasses.field(default_factory=dict)
    collision: str = "chm_mrt"        # or "srt2": single relaxation time, second-order EDF

    @property
    def shape(self):
        nz, ny, nx = self.mask.shape
        return nx, ny, nz

    @property
    def nu(self) -> float:
        return (self.tau - 0.5) / 3.0


def fluid_count(mask: np.ndarray) -> int:
    return int(np.count_nonzero(mask == FLUID))


# ---------------------------------------------------------------------------
# Config 1: straight periodic pipe (Poiseuille)
# ---------------------------------------------------------------------------

def pipe_case(nx: int = 64, ny: int = 24, nz: int = 24, radius: float = 10.0,
              center: tuple = (11.5, 11.5), g: float = 1e-6, tau: float = 0.8,
              steps: int = 2000) -> Case:
    """Circular pipe along x, periodic in x, walls elsewhere.

    With the defaults: 64x24x24, radius 10 lu centred at (11.5, 11.5),
    20,224 fluid nodes (316 per cross-section), body force 1e-6 along x.
    """
    y = np.arange(ny, dtype=np.float64)[:, None]
    z = np.arange(nz, dtype=np.float64)[None, :]
    inside = (y - center[0]) ** 2 + (z - center[1]) ** 2 < radius * radius  # [ny, nz]
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, :, :] = np.where(inside.T[:, :, None], FLUID, SOLID)
    return Case(name=f"pipe{nx}x{ny}x{nz}_R{radius:g}", mask=mask, periodic=PERIODIC_X,
                tau=tau, g=(g, 0.0, 0.0), steps=steps,
                meta=dict(radius=radius, center=center))


def open_pipe_case(nx: int = 48, ny: int = 14, nz: int = 14, radius: float = 5.0,
                   center: tuple = (6.5, 6.5), u_max: float = 0.01, tau: float = 0.8,
                   rho_out: float = 1.0) -> Case:
    """Straight circular pipe along x with a velocity inlet and a pressure
    outlet: the cells inside the radius on the x = 0 layer are inlet ghosts,
    on the x = nx - 1 layer outlet ghosts, the layers between are fluid and no
    axis is periodic.  The inlet carries the steady Poiseuille profile of
    centreline speed u_max (Womersley parameters with omega = 0)."""
    y = np.arange(ny, dtype=np.float64)[:, None]
    z = np.arange(nz, dtype=np.float64)[None, :]
    inside = ((y - center[0]) ** 2 + (z - center[1]) ** 2 < radius * radius).T   # [nz, ny]
    mask = np.zeros((nz, ny, nx), np.uint8)
    mask[:, :, 1:nx - 1] = np.where(inside[:, :, None], FLUID, SOLID)
    mask[:, :, 0] = np.where(inside, INLET, SOLID)
    mask[:, :, nx - 1] = np.where(inside, OUTLET, SOLID)
    nu = (tau - 0.5) / 3.0
    G0 = 4.0 * nu * u_max / (radius * radius)
    inlet = Inlet(axis=(1.0, 0.0, 0.0), center=(0.0, center[0], center[1]), radius=radius,
                  G0=G0, G1=0.0, omega=0.0)
    return Case(name=f"openpipe{nx}x{ny}x{nz}_R{radius:g}", mask=mask, periodic=0, tau=tau,
                rho_out=rho_out, inlet=inlet, meta=dict(radius=radius, center=center, u_max=u_max))


def periodic_box_case(nx: int, ny: int, nz: int, tau: float = 0.8, g=(0.0, 0.0, 0.0),
                      rates=(1.0, 1.0, 1.0, 1.0)) -> Case:
    """Fully periodic box with every node fluid."""
    mask = np.full((nz, ny, nx), FLUID, np.uint8)
    return Case(name=f"box{nx}x{ny}x{nz}", mask=mask,
                periodic=PERIODIC_X | PERIODIC_Y | PERIODIC_Z,
                tau=tau, g=tuple(g), rates=tuple(rates))


def channel_case(nx: int, ny: int, nz: int, tau: float, g: float) -> Case:
    """Planar channel: walls at the y = 0 and y = ny-1 layers, periodic x, z."""
    mask = np.full((nz, ny, nx), FLUID, np.uint8)
    mask[:, 0, :] = SOLID
    mask[:, ny - 1, :] = SOLID
    return Case(name=f"channel{nx}x{ny}x{nz}", mask=mask,
                periodic=PERIODIC_X | PERIODIC_Z, tau=tau, g=(g, 0.0, 0.0))


def random_tiny_case(seed: int, nx: int = 7, ny: int = 6, nz: int = 5) -> Case:
    """Small random mask with every cell type and random parameters.

    About 70 % of the cells are fluid; a few solid cells are turned into inlet
    and outlet ghost cells; periodic bits, relaxation rates in (0, 2), a body
    force and an oscillating inlet are drawn at random.
    """
    rng = np.random.default_rng(seed)
    mask = (rng.random((nz, ny, nx)) < 0.7).astype(np.uint8)
    ghosts = np.argwhere(mask == SOLID)
    rng.shuffle(ghosts)
    k = len(ghosts)
    for i, (z, y, x) in enumerate(ghosts[: max(2, k // 3)]):
        mask[z, y, x] = INLET if i % 2 == 0 else OUTLET
    if not np.any(mask == FLUID):
        mask[0, 0, 0] = FLUID
    periodic = int(rng.integers(0, 8))
    tau = float(rng.uniform(0.55, 1.6))
    rates = tuple(float(v) for v in rng.uniform(0.3, 1.9, 4))
    g = tuple(float(v) for v in rng.uniform(-1e-3, 1e-3, 3))
    ax = rng.normal(size=3)
    ax /= np.linalg.norm(ax)
    inlet = Inlet(axis=tuple(float(v) for v in ax),
                  center=(nx / 2.0, ny / 2.0, nz / 2.0), radius=float(max(nx, ny, nz)),
                  G0=float(rng.uniform(1e-5, 5e-5)), G1=float(rng.uniform(1e-5, 5e-5)),
                  omega=float(2 * math.pi / rng.integers(20, 60)))
    return Case(name=f"tiny{seed}", mask=mask, periodic=periodic, tau=tau, rates=rates,
                g=g, rho_out=float(rng.uniform(0.99, 1.01)), inlet=inlet, seed=seed)


# ---------------------------------------------------------------------------
# Configs 2-5: synthetic aneurysm family
# ---------------------------------------------------------------------------

# Reference geometry at the 256^3 size; every length scales with n / 256.
_TORUS_CENTER = (128.0, 100.0, 128.0)
_TORUS_MAJOR = 80.0
_TUBE_RADIUS = 12.0
_SAC_RADIUS = (18.0, 30.0)
_SAC_ANGLE_DEG = (80.0, 100.0)
# Womersley inlet at the 256^3 size: alpha = 3, period 4000 steps, tube radius
# 12 gives tau = 0.5 + 3 nu with nu = omega R^2 / alpha^2.
_WOMERSLEY_ALPHA = 3.0
_PERIOD_256 = 4000
# Steady centreline speed of the inlet profile (lattice units); with G1 = G0 the
# pulsatile peak centreline speed is close to 0.05.
_U_STEADY_CENTRE = 0.0329


def _sac_params(seed: int):
    rng = np.random.default_rng(seed)
    r_sac = float(rng.uniform(*_SAC_RADIUS))
    theta = math.radians(float(rng.uniform(*_SAC_ANGLE_DEG)))
    return r_sac, theta


def _aneurysm_mask(n: int, seed: int, tube_radius: Optional[float] = None,
                   ny: Optional[int] = None, nz: Optional[int] = None) -> tuple:
    """Voxelize the aneurysm geometry in an n^3 box (lengths scaled by n/256)."""
    s = n / 256.0
    nx = n
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    cx, cy, cz = (c * s for c in _TORUS_CENTER)
    rm = _TORUS_MAJOR * s
    rt = (_TUBE_RADIUS * s) if tube_radius is None else tube_radius
    r_sac0, theta = _sac_params(seed)
    r_sac = r_sac0 * s
    d_sac = (_TORUS_MAJOR + _TUBE_RADIUS + 0.4 * r_sac0) * s
    sx, sy, sz = cx + d_sac * math.cos(theta), cy + d_sac * math.sin(theta), cz
    mask = np.zeros((nz, ny, nx), np.uint8)

    def box(lo, hi, size):
        return max(0, int(math.floor(lo))), min(size, int(math.ceil(hi)) + 1)

    # half torus (y >= cy)
    z0, z1 = box(cz - rt, cz + rt, nz)
    y0, y1 = box(cy, cy + rm + rt, ny)
    x0, x1 = box(cx - rm - rt, cx + rm + rt, nx)
    zz, yy, xx = np.meshgrid(np.arange(z0, z1, dtype=np.float64),
                             np.arange(y0, y1, dtype=np.float64),
                             np.arange(x0, x1, dtype=np.float64), indexing="ij")
    rho = np.sqrt((xx - cx) ** 2 + (yy - cy) ** 2)
    inside = ((rho - rm) ** 2 + (zz - cz) ** 2 < rt * rt) & (yy >= cy)
    mask[z0:z1, y0:y1, x0:x1][inside] = FLUID
    del zz, yy, xx, rho, inside

    # two straight legs along y from the y = 0 layer up to the arc ends
    legs = ((cx + rm, INLET), (cx - rm, OUTLET))
    for lx, ghost in legs:
        xa, xb = box(lx - rt, lx + rt, nx)
        za, zb = box(cz - rt, cz + rt, nz)
        zz, xx = np.meshgrid(np.arange(za, zb, dtype=np.float64),
                             np.arange(xa, xb, dtype=np.float64), indexing="ij")
        disk = (xx - lx) ** 2 + (zz - cz) ** 2 < rt * rt          # [z, x]
        ytop = min(ny, int(math.floor(cy)) + 1)
        sub = mask[za:zb, 1:ytop, xa:xb]
        sub[np.broadcast_to(disk[:, None, :], sub.shape)] = FLUID
        g0 = mask[za:zb, 0, xa:xb]
        g0[disk] = ghost

    # spherical sac
    za, zb = box(sz - r_sac, sz + r_sac, nz)
    ya, yb = box(sy - r_sac, sy + r_sac, ny)
    xa, xb = box(sx - r_sac, sx + r_sac, nx)
    ya = max(ya, 1)
    zz, yy, xx = np.meshgrid(np.arange(za, zb, dtype=np.float64),
                             np.arange(ya, yb, dtype=np.float64),
                             np.arange(xa, xb, dtype=np.float64), indexing="ij")
    ball = (xx - sx) ** 2 + (yy - sy) ** 2 + (zz - sz) ** 2 < r_sac * r_sac
    mask[za:zb, ya:yb, xa:xb][ball] = FLUID
    geo = dict(scale=s, torus_center=(cx, cy, cz), major_radius=rm, tube_radius=rt,
               sac_radius=r_sac, sac_center=(sx, sy, sz), sac_angle_deg=math.degrees(theta),
               inlet_center=(cx + rm, 0.0, cz), outlet_center=(cx - rm, 0.0, cz))
    return mask, geo


def aneurysm_case(n: int = 256, seed: int = 0, period: Optional[int] = None,
                  tube_radius: Optional[float] = None, steps: Optional[int] = None,
                  u_steady_centre: float = _U_STEADY_CENTRE, tau: Optional[float] = None) -> Case:
    """Synthetic aneurysm in an n^3 box with a Womersley inlet and a zero-pressure outlet.

    Acoustic scaling (Sec. 3.4): all lengths scale with n/256, the period in
    steps scales with n/256 and the lattice velocity is unchanged, so tau - 1/2
    doubles when n doubles.  n = 256 gives tau = 0.575398 (period 4000),
    n = 512 gives tau = 0.650796 (period 8000), n = 128 gives 0.537699 (2000).
    ``tau`` overrides the relaxation time at the same inlet speed.
    """
    mask, geo = _aneurysm_mask(n, seed, tube_radius)
    rt = geo["tube_radius"]
    if period is None:
        period = int(round(_PERIOD_256 * n / 256.0))
    omega = 2.0 * math.pi / period
    if tau is None:
        nu = omega * rt * rt / (_WOMERSLEY_ALPHA ** 2)
        tau = 0.5 + 3.0 * nu
    else:
        # a given relaxation time (viscosity) at the same inlet speed; the
        # Womersley number then follows from it
        nu = (tau - 0.5) / 3.0
    G0 = 4.0 * nu * u_steady_centre / (rt * rt)
    inlet = Inlet(axis=(0.0, 1.0, 0.0), center=geo["inlet_center"], radius=rt,
                  G0=G0, G1=G0, omega=omega)
    if steps is None:
        steps = 5 * period
    return Case(name=f"aneurysm{n}_s{seed}", mask=mask, periodic=0, tau=tau,
                inlet=inlet, rho_out=1.0, steps=steps, period=period, seed=seed,
                meta=geo)


def batch_cases(first_seed: int = 1000, count: int = 48) -> list:
    """Uneven batch: cubic boxes L ~ U{64..192} (multiples of 8), fluid fraction
    ~U[5 %, 12 %] reached by bisection on the tube radius, tau ~ U[0.51, 1.0],
    Womersley alpha = 3 with each geometry's own viscosity and radius."""
    out = []
    for seed in range(first_seed, first_seed + count):
        rng = np.random.default_rng(seed)
        L = int(rng.integers(8, 25)) * 8
        frac = float(rng.uniform(0.05, 0.12))
        tau = float(rng.uniform(0.51, 1.0))
        lo, hi = 0.02 * L, 0.2 * L
        mask = geo = None
        for _ in range(18):
            mid = 0.5 * (lo + hi)
            mask, geo = _aneurysm_mask(L, seed, tube_radius=mid)
            f = fluid_count(mask) / float(L ** 3)
            if f < frac:
                lo = mid
            else:
                hi = mid
        mask, geo = _aneurysm_mask(L, seed, tube_radius=0.5 * (lo + hi))
        rt = geo["tube_radius"]
        nu = (tau - 0.5) / 3.0
        omega = _WOMERSLEY_ALPHA ** 2 * nu / (rt * rt)
        period = int(round(2 * math.pi / omega))
        G0 = 4.0 * nu * _U_STEADY_CENTRE / (rt * rt)
        inlet = Inlet(axis=(0.0, 1.0, 0.0), center=geo["inlet_center"], radius=rt,
                      G0=G0, G1=G0, omega=omega)
        out.append(Case(name=f"batch{seed}_L{L}", mask=mask, tau=tau, inlet=inlet,
                        period=period, seed=seed, meta=dict(geo, target_fraction=frac)))
    return out
