"""Stability of CHM-MRT against the SRT comparator (Sec. 2.1.2, Sec. 2.2.3).

The classical SRT operator with the second-order EDF becomes unusable at small
Fourier numbers Fo = nu dt / dx^2 (nu in lattice units), while the central
Hermite MRT operator keeps running; the paper's coarse run (tau 0.503, peak
lattice speed about 0.064) is one the SRT operator could not complete.  This
module steps a synthetic aneurysm with the Womersley inlet at a fixed inlet
speed and decreasing tau with both operators on the GPU and records, for each,
whether the run stays finite and bounded.

    python -m paper_2101_11107_amd.stability --n 128 --storage f32
"""

from __future__ import annotations

import math
import time

import numpy as np

from . import lbm

TAUS = (0.5377, 0.52, 0.515, 0.51, 0.505, 0.503, 0.5015, 0.501)


def run_one(case, collision: str, storage: str, steps: int, chunk: int = 200, u_limit: float = 0.3) -> dict:
    """Step ``case`` with one operator; stop at the first chunk whose monitors
    are not finite (the library reports LBM_EUNSTABLE) or whose largest speed
    exceeds ``u_limit``."""
    import dataclasses
    c = dataclasses.replace(case, collision=collision)
    dom = lbm.Domain(c, storage=storage)
    dom.init()
    done, status, umax = 0, "stable", 0.0
    t0 = time.perf_counter()
    try:
        while done < steps:
            k = min(chunk, steps - done)
            dom.step(k)
            done += k
            try:
                dom.monitors()
            except lbm.LbmError as e:
                if e.code != lbm.LBM_EUNSTABLE:
                    raise
                status = "non-finite"
                break
            _, u = dom.moments()
            umax = float(u.abs().max().item()) if u.numel() else 0.0
            if not math.isfinite(umax) or umax > u_limit:
                status = "diverged"
                break
    finally:
        dom.close()
    return {"collision": collision, "status": status, "steps": done, "u_max": umax,
            "seconds": round(time.perf_counter() - t0, 3)}


def sweep(n: int = 128, seed: int = 0, storage: str = "f32", taus=TAUS, steps: int = 4000,
          u_centre: float = 0.06) -> dict:
    """Both operators at every tau, with a steady parabolic inflow of centreline
    speed ``u_centre`` (the paper's coarse run: steady inflow, peak lattice
    speed about 0.064).  Returns the table and the smallest stable tau of each
    operator."""
    import dataclasses
    from synth import aneurysm_case
    rows = []
    for tau in taus:
        case = aneurysm_case(n, seed, tau=tau, u_steady_centre=u_centre)
        case = dataclasses.replace(case, inlet=dataclasses.replace(case.inlet, G1=0.0, omega=0.0))
        row = {"tau": tau, "fourier": round((tau - 0.5) / 3.0, 6), "steps": steps}
        for coll in ("chm_mrt", "srt2"):
            r = run_one(case, coll, storage, steps)
            row[coll] = {k: r[k] for k in ("status", "steps", "u_max")}
        rows.append(row)
    lowest = {}
    for coll in ("chm_mrt", "srt2"):
        ok = [r["tau"] for r in rows if r[coll]["status"] == "stable"]
        lowest[coll] = min(ok) if ok else None
    return {"n": n, "seed": seed, "storage": storage, "rows": rows, "lowest_stable_tau": lowest}


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="stability sweep: CHM-MRT against SRT")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--storage", default="f32")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--u-centre", type=float, default=0.06)
    a = ap.parse_args(argv)
    res = sweep(a.n, a.seed, a.storage, steps=a.steps, u_centre=a.u_centre)
    for r in res["rows"]:
        print(f"tau {r['tau']:.4f} Fo {r['fourier']:.5f}: CHM-MRT {r['chm_mrt']['status']:>10} "
              f"(u_max {r['chm_mrt']['u_max']:.4f}), SRT {r['srt2']['status']:>10} "
              f"(step {r['srt2']['steps']}, u_max {r['srt2']['u_max']:.4f})", flush=True)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
