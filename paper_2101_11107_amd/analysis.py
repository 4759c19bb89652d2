"""The paper's resolution study on a synthetic aneurysm (Sec. 3.2 and 3.4).

A high-resolution run (n^3) and a low-resolution run of the same geometry at
twice the grid spacing ((n/2)^3, acoustic scaling: the same lattice velocity,
half the steps per period) are stepped for several inlet periods on the GPU:

* three monitoring points around the sac record the velocity over all periods;
  the change of their signal from one period to the next shows when the flow
  no longer carries traces of the initial state (Sec. 3.2 samples the fourth
  cycle);
* the velocity averaged over the last period (inside the step kernel) is
  compared on three orthogonal planes through the sac centre: per plane the
  mean similarity index of Eq. (11), its histogram, and the joint histogram
  of the normalized speeds of both runs (Sec. 3.4);
* the wall-clock time of both runs gives the cost ratio (the paper quotes 14x
  for eight times fewer points and half the steps).

    python -m paper_2101_11107_amd.analysis --n 256 --cycles 4
"""

from __future__ import annotations

import time

import numpy as np

from . import lbm

PLANE_AXES = ("x", "y", "z")     # planes I, II, III: normal to x, y and z through the sac centre


def similarity_index_points(u_hr: np.ndarray, u_lr: np.ndarray) -> np.ndarray:
    """Eq. (11) per point, read with the factor 1/2 that maps it into [0, 1]:
    SI = (1 + cos) / 2 * (1 - | |a| / max|a| - |b| / max|b| |), maxima over the
    given points (one plane); points where either speed is zero take cos = 0.
    u_*: [m, 3]."""
    a = np.linalg.norm(u_hr, axis=1)
    b = np.linalg.norm(u_lr, axis=1)
    den = a * b
    cos = np.where(den > 0, (u_hr * u_lr).sum(axis=1) / np.where(den > 0, den, 1.0), 0.0)
    amax = a.max() if a.size and a.max() > 0 else 1.0
    bmax = b.max() if b.size and b.max() > 0 else 1.0
    return 0.5 * (1.0 + cos) * (1.0 - np.abs(a / amax - b / bmax))


def dense_field(u_nodes: np.ndarray, xyz: np.ndarray, shape) -> np.ndarray:
    """Nodal velocities [3, n] at cells xyz [n, 3] -> dense [nz, ny, nx, 3], zero
    off the fluid (the walls are at rest)."""
    nz, ny, nx = shape
    out = np.zeros((nz, ny, nx, 3))
    out[xyz[:, 2], xyz[:, 1], xyz[:, 0]] = u_nodes.T
    return out


def trilinear(dense: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Trilinear interpolation of a dense [nz, ny, nx, 3] field at points
    p [m, 3] = (x, y, z) in its own grid units (clamped to the box)."""
    nz, ny, nx, _ = dense.shape
    x = np.clip(p[:, 0], 0, nx - 1)
    y = np.clip(p[:, 1], 0, ny - 1)
    z = np.clip(p[:, 2], 0, nz - 1)
    x0 = np.minimum(np.floor(x).astype(np.int64), nx - 2 if nx > 1 else 0)
    y0 = np.minimum(np.floor(y).astype(np.int64), ny - 2 if ny > 1 else 0)
    z0 = np.minimum(np.floor(z).astype(np.int64), nz - 2 if nz > 1 else 0)
    fx, fy, fz = (x - x0)[:, None], (y - y0)[:, None], (z - z0)[:, None]
    x1, y1, z1 = np.minimum(x0 + 1, nx - 1), np.minimum(y0 + 1, ny - 1), np.minimum(z0 + 1, nz - 1)
    c = 0.0
    for zi, wz in ((z0, 1 - fz), (z1, fz)):
        for yi, wy in ((y0, 1 - fy), (y1, fy)):
            for xi, wx in ((x0, 1 - fx), (x1, fx)):
                c = c + wz * wy * wx * dense[zi, yi, xi]
    return c


def plane_points(mask: np.ndarray, axis: str, at: int) -> np.ndarray:
    """Fluid cells (x, y, z) of the plane normal to `axis` at index `at`."""
    zyx = np.argwhere(mask == 1)
    col = {"x": 2, "y": 1, "z": 0}[axis]
    sel = zyx[zyx[:, col] == at]
    return sel[:, ::-1].astype(np.int64)


def run_cycles(case, storage: str, cycles: int, probes: np.ndarray, every: int) -> dict:
    """Step `case` from rest for `cycles` periods; probes record every `every`
    steps; u is averaged over the last period inside the step kernel."""
    import torch
    d = lbm.Domain(case, storage=storage)
    d.init()
    d.set_probes(probes, every=every, capacity=cycles * case.period // every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d.step((cycles - 1) * case.period)
    d.average(lbm.LBM_AVG_RESET)
    d.average(lbm.LBM_AVG_TRACK)
    d.step(case.period)
    u_avg = d.average(lbm.LBM_AVG_READ)
    d.stream.synchronize()
    seconds = time.perf_counter() - t0
    out = {"u_avg": u_avg.cpu().numpy(), "xyz": d.coords(), "probes": d.probe_records().cpu().numpy(),
           "seconds": seconds, "steps": cycles * case.period}
    d.close()
    return out


def periodicity(records: np.ndarray, per_cycle: int) -> list:
    """Per cycle from the second on: the largest change of the probe speeds
    against the previous cycle, relative to the largest probe speed."""
    speed = np.linalg.norm(records[:, :, 1:], axis=2)              # [t, probe]
    ncyc = speed.shape[0] // per_cycle
    ref = max(float(speed.max()), 1e-300)
    return [float(np.abs(speed[k * per_cycle:(k + 1) * per_cycle] - speed[(k - 1) * per_cycle:k * per_cycle]).max()
                  / ref) for k in range(1, ncyc)]


def resolution_study(seed: int = 48, n: int = 256, cycles: int = 4, storage: str = "f32",
                     samples_per_cycle: int = 100, bins: int = 20) -> dict:
    from synth import aneurysm_case
    hr_case = aneurysm_case(n, seed)
    lr_case = aneurysm_case(n // 2, seed)
    geo = hr_case.meta
    sx, sy, sz = geo["sac_center"]
    rs = geo["sac_radius"]
    # three points around the sac: its centre and half a radius towards the
    # parent vessel and across it
    pts_hr = np.array([[sx, sy, sz], [sx, sy - 0.5 * rs, sz], [sx + 0.5 * rs, sy, sz]])
    probes_hr = np.rint(pts_hr).astype(np.int32)
    probes_lr = np.rint(pts_hr / 2.0).astype(np.int32)
    for p, m in ((probes_hr, hr_case.mask), (probes_lr, lr_case.mask)):
        for q in p:
            if m[q[2], q[1], q[0]] != 1:
                raise ValueError(f"probe {q.tolist()} is not in the fluid")
    hr = run_cycles(hr_case, storage, cycles, probes_hr, hr_case.period // samples_per_cycle)
    lr = run_cycles(lr_case, storage, cycles, probes_lr, lr_case.period // samples_per_cycle)
    hr_dense = dense_field(hr["u_avg"], hr["xyz"], hr_case.mask.shape)
    lr_dense = dense_field(lr["u_avg"], lr["xyz"], lr_case.mask.shape)
    planes = []
    for axis, at in zip(PLANE_AXES, (sx, sy, sz)):
        pts = plane_points(hr_case.mask, axis, int(round(at)))
        u_hr = hr_dense[pts[:, 2], pts[:, 1], pts[:, 0]]
        u_lr = trilinear(lr_dense, pts / 2.0)       # the same physical point in the coarse grid
        si = similarity_index_points(u_hr, u_lr)
        a = np.linalg.norm(u_hr, axis=1)
        b = np.linalg.norm(u_lr, axis=1)
        hist_si, _ = np.histogram(si, bins=bins, range=(0.0, 1.0))
        joint, _, _ = np.histogram2d(b / max(b.max(), 1e-300), a / max(a.max(), 1e-300), bins=bins,
                                     range=((0, 1), (0, 1)))
        planes.append({"plane": axis, "at": int(round(at)), "points": int(len(pts)),
                       "similarity_index": float(si.mean()),
                       "si_histogram": (hist_si / max(len(si), 1)).round(5).tolist(),
                       "speed_joint_histogram_lr_x_hr_y": (joint / max(len(si), 1)).round(5).tolist()})
    return {"seed": seed, "n_high": n, "n_low": n // 2, "cycles": cycles, "storage": storage,
            "steps_high": hr["steps"], "steps_low": lr["steps"],
            "fluid_nodes_high": int(hr["xyz"].shape[0]), "fluid_nodes_low": int(lr["xyz"].shape[0]),
            "seconds_high": round(hr["seconds"], 4), "seconds_low": round(lr["seconds"], 4),
            "cost_ratio": round(hr["seconds"] / lr["seconds"], 2),
            "periodicity_high": [round(v, 5) for v in periodicity(hr["probes"], samples_per_cycle)],
            "periodicity_low": [round(v, 5) for v in periodicity(lr["probes"], samples_per_cycle)],
            "planes": planes}


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="resolution study: planes, similarity index, monitoring points")
    ap.add_argument("--seed", type=int, default=48)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--cycles", type=int, default=4)
    ap.add_argument("--storage", default="f32")
    a = ap.parse_args(argv)
    res = resolution_study(a.seed, a.n, a.cycles, a.storage)
    for p in res["planes"]:
        print(f"plane {p['plane']} = {p['at']}: {p['points']} points, SI {p['similarity_index']:.4f}", flush=True)
    print(f"periodicity (high) {res['periodicity_high']}, (low) {res['periodicity_low']}; "
          f"cost ratio {res['cost_ratio']}", flush=True)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
