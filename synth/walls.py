"""Wall links and wall distances of the synthetic geometries.

Input data for curved walls (Sec. 2.1.4): for every link from a fluid cell x
in a direction a whose neighbour x + c_a is a wall, the fraction q of the link
from x to the wall surface.  The surfaces are the analytic shapes the masks
are voxelized from, so q is found by bisection on the same predicate that
decides which cells are fluid.  No lattice Boltzmann arithmetic lives here.
"""

from __future__ import annotations

import math

import numpy as np

from .geometry import FLUID, SOLID, Case

# D3Q27 direction a = 9 (cz + 1) + 3 (cy + 1) + (cx + 1)
_C = np.array([(a % 3 - 1, (a // 3) % 3 - 1, a // 9 - 1) for a in range(27)], np.int64)


def wall_links(mask: np.ndarray, periodic: int) -> np.ndarray:
    """int32 [m, 4] = (x, y, z, a): fluid cell (x, y, z) and a direction a
    whose cell x + c_a is SOLID or lies outside a non-periodic box; x-fastest
    cell order, then a."""
    nz, ny, nx = mask.shape
    dims = (nx, ny, nz)
    fz, fy, fx = np.nonzero(mask == FLUID)
    cells = np.stack([fx, fy, fz], axis=1).astype(np.int64)      # sorted z, y, x -> x fastest
    out = []
    for a in range(27):
        if a == 13:
            continue
        p = cells + _C[a][None, :]
        inside = np.ones(len(p), bool)
        for ax in range(3):
            if (periodic >> ax) & 1:
                p[:, ax] %= dims[ax]
            else:
                inside &= (p[:, ax] >= 0) & (p[:, ax] < dims[ax])
        wall = ~inside
        ok = np.nonzero(inside)[0]
        wall[ok] = mask[p[ok, 2], p[ok, 1], p[ok, 0]] == SOLID
        k = np.nonzero(wall)[0]
        out.append(np.concatenate([cells[k], np.full((len(k), 1), a)], axis=1))
    links = np.concatenate(out, axis=0) if out else np.zeros((0, 4), np.int64)
    # x-fastest cell order, then direction
    key = ((links[:, 2] * ny + links[:, 1]) * nx + links[:, 0]) * 27 + links[:, 3]
    return np.ascontiguousarray(links[np.argsort(key, kind="stable")], np.int32)


def fluid_predicate(case: Case):
    """Continuous form of the fluid test that voxelized ``case.mask``:
    a function of float arrays (x, y, z) -> bool array.  Pipe and aneurysm
    cases only."""
    meta = case.meta
    if "radius" in meta and "center" in meta:             # straight pipe along x
        cy, cz = meta["center"]
        r2 = meta["radius"] ** 2

        def pipe(x, y, z):
            return (y - cy) ** 2 + (z - cz) ** 2 < r2
        return pipe
    if "torus_center" in meta:                               # aneurysm
        cx, cy, cz = meta["torus_center"]
        rm, rt = meta["major_radius"], meta["tube_radius"]
        sx, sy, sz = meta["sac_center"]
        rs = meta["sac_radius"]
        legs = (cx + rm, cx - rm)

        def aneurysm(x, y, z):
            rho = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
            f = ((rho - rm) ** 2 + (z - cz) ** 2 < rt * rt) & (y >= cy)
            # legs: grid rows 1 .. floor(cy); their inlet/outlet plane lies at y = 1/2
            for lx in legs:
                f |= ((x - lx) ** 2 + (z - cz) ** 2 < rt * rt) & (y > 0.5) & (y <= math.floor(cy))
            f |= ((x - sx) ** 2 + (y - sy) ** 2 + (z - sz) ** 2 < rs * rs) & (y >= 1.0)
            return f
        return aneurysm
    raise ValueError(f"{case.name}: no analytic surface known")


def wall_distances(case: Case, links: np.ndarray, iters: int = 60) -> np.ndarray:
    """q [m] in (0, 1] for each link (x, y, z, a): the fraction of the link
    from the node to where ``fluid_predicate`` turns false, by bisection.
    Links whose ends do not straddle the surface (a cell made solid by the box
    and not by the shape) get q = 1/2."""
    pred = fluid_predicate(case)
    p0 = links[:, :3].astype(np.float64)
    c = _C[links[:, 3]].astype(np.float64)
    lo = np.zeros(len(links))
    hi = np.ones(len(links))
    ok = pred(*(p0.T)) & ~pred(*((p0 + c).T))
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        pm = p0 + mid[:, None] * c
        inside = pred(pm[:, 0], pm[:, 1], pm[:, 2])
        lo = np.where(inside, mid, lo)
        hi = np.where(inside, hi, mid)
    q = np.where(ok, hi, 0.5)
    return np.clip(q, 1e-12, 1.0)


def random_wall_distances(links: np.ndarray, seed: int, lo: float = 0.02, hi: float = 1.0) -> np.ndarray:
    """Seeded q ~ U[lo, hi] per link (for geometries without an analytic surface)."""
    return np.random.default_rng(seed).uniform(lo, hi, len(links))
