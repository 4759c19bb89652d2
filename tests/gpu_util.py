"""Helpers shared by the GPU tests: run the library and the oracle on one case."""

import numpy as np

W = np.array([(1 / 6 if cx else 2 / 3) * (1 / 6 if cy else 2 / 3) * (1 / 6 if cz else 2 / 3)
              for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)])
C = np.array([(cx, cy, cz) for cz in (-1, 0, 1) for cy in (-1, 0, 1) for cx in (-1, 0, 1)], np.float64)


def oracle_order(coords, mask):
    """Permutation taking library node order to the oracle's x-fastest order."""
    nz, ny, nx = mask.shape
    key = (coords[:, 2].astype(np.int64) * ny + coords[:, 1]) * nx + coords[:, 0]
    return np.argsort(key, kind="stable")


def gpu_run(case, storage, steps, device="cuda:0", wall_q=None):
    """Run the HIP path; return (domain, shifted post-collision populations [n, 27]
    as FP64, in the oracle's x-fastest node order).  wall_q: optional
    (links [m, 4], q [m]) for curved walls."""
    import torch
    from paper_2101_11107_amd import lbm
    dom = lbm.Domain(case, storage=storage, device=device, wall_q=wall_q)
    dom.init()
    if steps:
        dom.step(steps)
    f = dom.populations().cpu().numpy().T.copy()
    torch.cuda.synchronize()
    perm = oracle_order(dom.coords(), case.mask)
    return dom, f[perm]


def oracle_post(case, steps, nthreads=16, wall_q=None, long_double=False):
    """Oracle tier O2: shifted post-collision populations f*(steps) - w and u(steps).
    wall_q: optional (links [m, 4], q [m]) for curved walls.  long_double: run
    the long-double build of the same oracle (its double build holds unshifted
    populations of about 0.3, whose rounding reaches 1e-12 of the velocity of
    the config-1 pipe in 2000 steps); results are returned as FP64."""
    from oracle import o2
    wq = None if wall_q is None else {tuple(int(v) for v in lk): float(q)
                                      for lk, q in zip(wall_q[0], wall_q[1])}
    sim = o2.O2Sim(case, nthreads=nthreads, wall_q=wq, long_double=long_double)
    if steps:
        sim.run(steps)
    rho, u = sim.macroscopic()
    sim.collide()
    w = o2._weights(sim.real)
    fhat = np.asarray(sim.fpost - w[None, :], np.float64)
    return sim, fhat, np.asarray(rho, np.float64), np.asarray(u, np.float64)


def moments_from_post(fhat, g):
    """rho, u of the pre-collision state from shifted post-collision populations."""
    rho = 1.0 + fhat.sum(axis=1)
    j = fhat @ C
    u = (j - 0.5 * rho[:, None] * np.asarray(g, np.float64)[None, :]) / rho[:, None]
    return rho, u


def eps_u(u_gpu, u_ref):
    return float(np.max(np.abs(u_gpu - u_ref)) / np.max(np.abs(u_ref)))
