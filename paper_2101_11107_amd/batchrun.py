"""Batched stepping of the 48 uneven synthetic geometries with a fixed
execution configuration, for kernel traces and counter runs of the batch
kernel (the bench's batch leg autotunes instead).

    python -m paper_2101_11107_amd.batchrun --storage f16s --config 0,256,0,0,192 --row-tile 16

prints one JSON line: nodes, steps, time per step and the algorithmic
bandwidth (54 populations per node and step).
"""

from __future__ import annotations

import argparse
import json
import sys
import time


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--storage", default="f16s", choices=["f64", "f32", "f16s", "bf16s"])
    ap.add_argument("--config", default="0,256,0,0,192",
                    help="mode,block,stream_store,grid,group_mb (lbm_batch_set_config)")
    ap.add_argument("--row-tile", type=int, default=16)
    ap.add_argument("--steps", type=int, default=160)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    a = ap.parse_args(argv)
    import torch
    import synth
    from . import lbm

    if a.copy_probe_mib:
        src = torch.empty(a.copy_probe_mib << 20, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cfg = [int(v) for v in a.config.split(",")]
    doms = [lbm.Domain(c, storage=a.storage, device="cuda:0", row_tile=a.row_tile) for c in synth.batch_cases()]
    for d in doms:
        d.init()
    n = sum(d.n for d in doms)
    b = lbm.Batch(doms)
    b.set_config(cfg)
    b.step(a.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(a.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.status()
    b.close()
    for d in doms:
        d.close()
    pop = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}[a.storage]
    us = dt * 1e6 / a.steps
    print(json.dumps({"workload": "batch48_uneven", "storage": a.storage, "config": cfg, "row_tile": a.row_tile,
                      "fluid_nodes": n, "steps": a.steps, "us_per_step": round(us, 2),
                      "algorithmic_TBs": round(54 * pop * n / (us * 1e-6) / 1e12, 3)}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
