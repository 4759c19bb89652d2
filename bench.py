"""Benchmark of the D3Q27 CHM-MRT step on one MI355X.

Default workload: the 512^3 synthetic aneurysm (seed 0: torus arc of major
radius 160 and tube radius 24 with a seeded sac, Womersley inlet with alpha = 3
and an 8000-step period, zero-pressure outlet, tau = 0.6508), shifted
populations stored in FP32: a 0.92 GB population working set, well beyond the
256 MB Infinity Cache, so the step runs against HBM.  The 256^3 geometry
(working set 0.11 GB, cache resident) is reported beside it.  A step is one fused stream-collide launch over
every fluid node (with its monitor partials); K steps are timed with HIP events
on the library's stream after W warm-up steps, inputs resident in HBM.

Prints one JSON line: fluid-node MLUPS, the roofline of the step kernel
(algorithmic bytes 54 populations x storage bytes per node update), the FP64
CPU oracle timed on a bounded sample on the host cores, and (``also``) the
other storage forms and the 512^3 geometry with their velocity error against
the FP64 run of the same geometry, the batch of 48 uneven geometries, and the
learned coarse-to-fine corrector (a reduced training protocol) with its
velocity error against the FP64 fine run beside the trilinear upsampling.
"""

import argparse
import dataclasses
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                 # MI355X HBM3E, 8 TB/s
POP_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
STEP_KERNEL = "k_step"


def kernel_source_hash():
    from paper_2101_11107_amd.profsum import kernel_source_hash as h
    return h()


def read_profile(storage, workload):
    """Values of the committed rocprofv3 summary for this kernel and workload,
    if it was taken on the current kernel source; {} otherwise."""
    path = os.path.join(ROOT, "profiles", f"traffic_{STEP_KERNEL}_{storage}_{workload}.txt")
    if not os.path.exists(path):
        return {}
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return {}
    return vals


def read_traffic(storage, workload):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated) or None."""
    try:
        return float(read_profile(storage, workload)["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# Untimed steps from rest before the warm-up (--spinup).  At rest the shifted
# populations are exactly zero, and for the first ~1000 steps, until the
# inlet's pressure wave has crossed the 512^3 domain, the in-place step runs
# faster than on the developed flow (data-dependent; the pull step does not
# change).  Timing starts on the developed flow.
SPINUP = 1000


def run_form(torch, lbm, case, storage, warmup, steps, want_u=False, wall_q=None, streaming="auto"):
    dom = lbm.Domain(case, storage=storage, device="cuda:0", wall_q=wall_q, streaming=streaming)
    dom.init()
    dom.step(SPINUP + warmup)
    dom.stream.synchronize()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(dom.stream)
    dom.step(steps)
    ev1.record(dom.stream)
    ev1.synchronize()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    mon = dom.monitors()
    out = dict(n=dom.n, ms=ms, ms_per_step=ms / steps, mlups=dom.n * steps / (ms * 1e-3) / 1e6,
               monitors=mon, streaming="inplace" if dom.in_place() else "pull")
    if want_u:
        _, u = dom.moments()
        out["u"] = u.cpu().numpy()
    dom.close()
    del dom
    torch.cuda.empty_cache()
    return out


def curved_bench(torch, lbm, case, storage, warmup, steps, plain, plain_pull):
    """Curved walls (interpolated bounce-back with the exact wall distance on
    every wall link of the geometry): the step rate against the plain halfway
    form of the same run with the same streaming pattern (and against the
    halfway pull run), and the pipe Poiseuille error of both wall rules against
    the start-up series at R = 5, 10, 20 (FP64, 20 R^2 steps)."""
    import numpy as np
    import scipy.special
    import synth
    links = synth.wall_links(case.mask, case.periodic)
    q = synth.wall_distances(case, links)
    r = run_form(torch, lbm, case, storage, warmup, steps, want_u=True, wall_q=(links, q))
    rf = roofline(r["n"], r["ms_per_step"], storage, None)
    out = {"workload": case.name.split("_")[0] + "_curved_walls", "storage": storage, "wall_links": int(len(links)),
           "mlups": round(r["mlups"], 1), "roofline_frac": rf["frac"], "streaming": r["streaming"],
           "rate_vs_halfway": round(r["mlups"] / plain["mlups"], 3),
           "rate_vs_halfway_pull": round(r["mlups"] / plain_pull["mlups"], 3)}
    if "u" in plain:
        out["u_rel_l2_vs_halfway"] = rel_l2(r["u"], plain["u"])
    lam = scipy.special.jn_zeros(0, 60)
    errs = {"halfway": [], "curved": []}
    for R in (5, 10, 20):
        n = int(2 * R + 4)
        pc = synth.pipe_case(nx=4, ny=n, nz=n, radius=R, center=((n - 1) / 2 + 0.3, (n - 1) / 2 - 0.2))
        pl = synth.wall_links(pc.mask, pc.periodic)
        pq = synth.wall_distances(pc, pl)
        nsteps = int(20 * R * R)
        cy, cz = pc.meta["center"]
        for kind, wq in (("halfway", None), ("curved", (pl, pq))):
            dom = lbm.Domain(pc, storage="f64", device="cuda:0", wall_q=wq)
            dom.init()
            dom.step(nsteps)
            _, u = dom.moments()
            u = u.cpu().numpy()
            xyz = dom.coords()
            dom.close()
            rr = np.sqrt((xyz[:, 1] - cy) ** 2 + (xyz[:, 2] - cz) ** 2)
            nu, g = pc.nu, pc.g[0]
            ua = g * (R * R - rr * rr) / (4 * nu)
            for lv in lam:
                ua = ua - 2 * g * R * R / nu * scipy.special.j0(lv * rr / R) / (lv ** 3 * scipy.special.j1(lv)) \
                    * np.exp(-lv * lv * nu * nsteps / (R * R))
            errs[kind].append(float(np.sqrt(((u[0] - ua) ** 2).sum() / (ua ** 2).sum())))
    out["pipe_l2_error_R5_10_20"] = {k: [round(e, 7) for e in v] for k, v in errs.items()}
    out["pipe_order"] = {k: round(float(np.log2(v[1] / v[2])), 2) for k, v in errs.items()}
    return out


def batch_bench(torch, lbm, steps, storage="f16s"):
    """48 uneven synthetic geometries (boxes 64^3..192^3, 5-12 % fluid, tau in
    [0.51, 1]) stepped together by the autotuned batch against the same domains
    stepped one after another (each with its own graph replays)."""
    import synth
    cases = synth.batch_cases()
    # the autotuner times every execution choice of the batch for each
    # row-tile edge of the node order and keeps the fastest
    b, doms, tile, tuned_ms, tile_ms = lbm.autotune_batch(cases, storage, row_tiles=(4, 8, 16), trial_steps=32)
    total = sum(d.n for d in doms)
    cfg = b.config()
    b.step(32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    b.status()
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    for d in doms:
        d.step(16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in doms:
        d.step(steps)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    b.close()
    for d in doms:
        d.close()
    del doms
    torch.cuda.empty_cache()
    ms = t_batch * 1e3 / steps
    return {"workload": "batch48_uneven", "storage": storage, "domains": len(cases), "fluid_nodes": total,
            "steps": steps, "batched_mlups": round(total * steps / t_batch / 1e6, 1),
            "sequential_mlups": round(total * steps / t_seq / 1e6, 1),
            "batched_over_sequential": round(t_seq / t_batch, 3),
            "autotuned_config": {"mode": ["launch_per_step", "persistent", "launch_per_step_in_place"][cfg[0]],
                                 "block": cfg[1],
                                 "stream_store": cfg[2], "grid": cfg[3], "group_mb": cfg[4], "row_tile": tile},
            "autotune_best_ms_per_step_by_row_tile": {str(k): round(v, 4) for k, v in tile_ms.items()},
            "autotune_best_ms_per_step": round(tuned_ms, 4),
            "roofline_frac": roofline(total, ms, storage, None)["frac"]}


def corrector_bench():
    """The learned corrector's protocol: 48 training geometries, 6000 Adam
    steps, 16 held-out geometries scored against their FP64 fine runs, with
    the fallback thresholds calibrated on the training geometries."""
    import numpy as np
    from paper_2101_11107_amd import corrector as C
    res = C.run_protocol(range(48), range(48, 64), C.TrainConfig(iters=6000, log_every=1500),
                         log=lambda m: note(f"corrector: {m}"))
    l2n, l2t = np.array(res["l2_net"]), np.array(res["l2_tri"])
    sin, sit = np.array(res["si_net"]), np.array(res["si_tri"])
    return {"workload": "corrector_aneurysm128_to_256", "train_geometries": 48, "held_out_geometries": 16,
            "adam_steps": res["train_iters"], "train_seconds": round(res["train_seconds"], 2),
            "ms_per_train_step": round(1e3 * res["train_seconds"] / res["train_iters"], 2),
            "data_seconds": round(res["data_seconds"], 2),
            "u_rel_l2_net_vs_f64_fine": round(float(l2n.mean()), 5),
            "u_rel_l2_trilinear_vs_f64_fine": round(float(l2t.mean()), 5),
            "similarity_index_net": round(float(sin.mean()), 5),
            "similarity_index_trilinear": round(float(sit.mean()), 5),
            "held_out_better_on_both": int(np.sum((l2n < l2t) & (sin > sit))),
            "fallback_rate": res["fallback_rate"],
            "coarse_run_s": round(res["coarse_seconds"], 4),
            "inference_s": round(res["infer_seconds"], 4),
            "fine_run_f32_s": round(res["fine_seconds_f32"], 4),
            "fine_run_f64_s": round(res["fine_seconds_f64"], 4),
            "speedup_vs_fine_f32": round(res["speedup_vs_fine_f32"], 2)}


def roofline(n, ms_per_step, storage, traffic, wall_links=0):
    # algorithmic bytes per launch: 54 populations per node, plus one
    # curved-wall weight per wall link (8 B with FP64 storage, 4 B otherwise)
    alg = 54 * POP_BYTES[storage] * n + (8 if storage == "f64" else 4) * wall_links
    achieved = alg / (ms_per_step * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "algorithmic_bytes_per_launch": alg}


def host_threads():
    """Threads the host gives this process: its CPU affinity, capped by
    OMP_NUM_THREADS when the environment sets it (a shared GPU host allots a
    fixed CPU share per GPU that way)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_ORACLE_TIMER = r"""
import json, sys, time
sys.path.insert(0, sys.argv[1])
import synth
from oracle import o2
size, threads, budget = int(sys.argv[2]), int(sys.argv[3]), float(sys.argv[4])
case = synth.aneurysm_case(size, seed=0)
sim = o2.O2Sim(case, nthreads=threads)
sim.run(1)
# each call ends with a serial mass and momentum sum: size the timed call
# from the difference of a one-step and a three-step call, and time all its
# steps in one call
t0 = time.perf_counter()
sim.run(1)
t1 = time.perf_counter()
sim.run(3)
per_step = max(1e-6, 0.5 * ((time.perf_counter() - t1) - (t1 - t0)))
steps = max(2, int(budget / per_step))
t0 = time.perf_counter()
sim.run(steps)
print(json.dumps({"n": sim.n, "steps": steps, "seconds": time.perf_counter() - t0, "name": case.name}))
"""


def _time_oracle(size, threads, budget_s):
    """Step the oracle from rest for about budget_s seconds in a child
    process that loads neither torch nor the GPU library (their idle worker
    threads would compete with the oracle's for the host cores)."""
    import subprocess
    res = subprocess.run([sys.executable, "-c", _ORACLE_TIMER, ROOT, str(size), str(threads), str(budget_s)],
                         capture_output=True, text=True, check=True, timeout=600)
    return json.loads(res.stdout.strip().splitlines()[-1])


def cpu_baseline(size, budget_s):
    """Oracle tier O2 (FP64, C with OpenMP) on the same aneurysm geometry,
    stepped from rest for about budget_s seconds on every host thread this
    process may use, then for about budget_s / 2 seconds on one thread."""
    from oracle import o2
    o2.build(force=False)
    threads = host_threads()
    r = _time_oracle(size, threads, budget_s)
    r1 = _time_oracle(size, 1, 0.5 * budget_s)
    return {"value": round(r["n"] * r["steps"] / r["seconds"] / 1e6, 3), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{r['name']}: {r['steps']} steps of the FP64 C/OpenMP oracle from rest "
                      f"({r['n']} fluid nodes, {r['seconds']:.1f} s, {threads} threads); "
                      f"{r1['steps']} steps on 1 thread ({r1['seconds']:.1f} s)",
            "single_thread_value": round(r1["n"] * r1["steps"] / r1["seconds"] / 1e6, 3),
            "cpu_model": cpu_model(), "host_cpu_count": os.cpu_count()}


def rel_l2(u, ref):
    import numpy as np
    return float(np.sqrt(((u - ref) ** 2).sum() / (ref ** 2).sum()))


def note(msg):
    """Progress line on stderr (stdout carries only the result line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    global SPINUP
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--storage", default="f32", choices=list(POP_BYTES))
    ap.add_argument("--workload", default="aneurysm512", choices=["aneurysm256", "aneurysm512"],
                    help="geometry of the timed run (the 256^3 one is Infinity Cache resident)")
    ap.add_argument("--walls", default="halfway", choices=["halfway", "curved"],
                    help="wall rule of the timed run: halfway bounce-back, or interpolated bounce-back with the "
                         "exact wall distance on every wall link (Eq. (9)-(10))")
    ap.add_argument("--spinup", type=int, default=SPINUP,
                    help="untimed steps from rest before the warm-up (every timed run)")
    ap.add_argument("--streaming", default="auto", choices=["auto", "pull", "inplace"],
                    help="streaming pattern of the timed run (lbm_set_streaming; auto picks by size)")
    ap.add_argument("--no-extra", action="store_true", help="skip the other storage forms and sizes")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-corrector", action="store_true", help="skip the learned-corrector protocol")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    args = ap.parse_args()
    SPINUP = max(0, args.spinup)
    if args.walls == "curved" and not args.no_extra:
        ap.error("--walls curved times the curved-wall step alone: add --no-extra")
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the method's multi-GPU "
              "decomposition is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import synth
    from paper_2101_11107_amd import lbm

    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    size = 256 if args.workload == "aneurysm256" else 512
    case = synth.aneurysm_case(size, seed=0)
    wall_q, nlinks = None, 0
    workload = args.workload
    if args.walls == "curved":
        links = synth.wall_links(case.mask, case.periodic)
        wall_q, nlinks = (links, synth.wall_distances(case, links)), int(len(links))
        workload += "_curved"
    main_run = run_form(torch, lbm, case, args.storage, args.warmup, args.steps, want_u=not args.no_extra,
                        wall_q=wall_q, streaming=args.streaming)
    note(f"{workload} {args.storage} ({main_run['streaming']} streaming): {main_run['mlups']:.1f} MLUPS, "
         f"{main_run['ms_per_step'] * 1e3:.2f} us per step")
    traffic = read_traffic(args.storage, workload)
    line = {
        "metric": "fluid-node MLUPS (D3Q27 CHM-MRT fused stream-collide step)",
        "value": round(main_run["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}_seed0_womersley_alpha3_period{case.period}", "box": [size] * 3,
                   "fluid_nodes": main_run["n"], "storage": args.storage, "tau": round(case.tau, 6),
                   "steps_per_graph": 16, "walls": args.walls, "streaming": main_run["streaming"],
                   "spinup_steps": SPINUP},
        "roofline": roofline(main_run["n"], main_run["ms_per_step"], args.storage, traffic, nlinks),
    }
    if nlinks:
        line["config"]["wall_links"] = nlinks
    prof = read_profile(args.storage, workload)
    if prof.get("avg_step_kernel_us"):
        # kernel-only average of the committed rocprofv3 trace (the event figure
        # above also contains the short gaps between graph-launched kernels)
        line["roofline"]["rocprof_avg_step_kernel_us"] = float(prof["avg_step_kernel_us"])
    mon = main_run["monitors"]
    line["monitors_last_step"] = {"mass": mon[0], "inlet_flux": mon[7], "outlet_flux": mon[8], "t": mon[9]}

    if not args.no_extra:
        also = []
        # the same run with the other streaming pattern (same values, other
        # places between steps)
        other = "pull" if main_run["streaming"] == "inplace" else "inplace"
        alt = run_form(torch, lbm, case, args.storage, args.warmup, args.steps, want_u=True, streaming=other)
        also.append({"workload": workload, "storage": args.storage, "streaming": other,
                     "mlups": round(alt["mlups"], 1),
                     "roofline_frac": roofline(alt["n"], alt["ms_per_step"], args.storage, None)["frac"],
                     "rate_vs_value": round(alt["mlups"] / main_run["mlups"], 3),
                     "velocity_bitwise_equal": bool(np.array_equal(alt["u"], main_run["u"]))})
        note(f"{other} streaming: {alt['mlups']:.1f} MLUPS")
        pull_run = alt if other == "pull" else main_run
        # every storage form at both geometries, velocity error and mass drift
        # against the FP64 run of the same geometry after the same steps
        for wl in (workload, "aneurysm256" if workload == "aneurysm512" else "aneurysm512"):
            sz = 256 if wl == "aneurysm256" else 512
            cs = case if wl == workload else synth.aneurysm_case(sz, seed=0)
            warm, steps_x = (args.warmup, args.steps) if wl == workload else (100, 1000)
            ref = run_form(torch, lbm, cs, "f64", warm, steps_x, want_u=True)
            note(f"{wl} f64: {ref['mlups']:.1f} MLUPS")
            if wl == workload:
                line["f32_velocity_rel_l2_vs_f64" if args.storage == "f32" else
                     f"{args.storage}_velocity_rel_l2_vs_f64"] = rel_l2(main_run["u"], ref["u"])
            for st in ("f64", "f32", "f16s", "bf16s"):
                if wl == workload and st == args.storage:
                    continue
                r = ref if st == "f64" else run_form(torch, lbm, cs, st, warm, steps_x, want_u=True)
                if st != "f64":
                    note(f"{wl} {st}: {r['mlups']:.1f} MLUPS")
                rf = roofline(r["n"], r["ms_per_step"], st, read_traffic(st, wl))
                row = {"workload": wl, "storage": st, "fluid_nodes": r["n"], "mlups": round(r["mlups"], 1),
                       "achieved_GBs": rf["achieved"], "roofline_frac": rf["frac"], "traffic": rf["traffic"],
                       "steps": SPINUP + warm + steps_x}
                if wl == "aneurysm256":
                    row["note"] = "populations fit in the 256 MB Infinity Cache"
                if st != "f64":
                    row["u_rel_l2_vs_f64"] = rel_l2(r["u"], ref["u"])
                    row["mass_drift_vs_f64"] = abs(r["monitors"][0] - ref["monitors"][0]) / ref["monitors"][0]
                also.append(row)
            del ref
        # the 512^3 configuration over its full length (five inlet periods):
        # every storage form against the FP64 run
        from paper_2101_11107_amd import precision
        case512 = case if workload == "aneurysm512" else synth.aneurysm_case(512, seed=0)
        ps = precision.study(case512, 40000)
        also.append({"workload": "aneurysm512_full_length_storage_forms", "steps": ps["steps"],
                     "average_steps": ps["average_steps"],
                     "vs_f64": {st: {k: (round(v, 10) if isinstance(v, float) else v) for k, v in ps[st].items()}
                                for st in ("f32", "f16s", "bf16s")}})
        note(f"precision study 40000 steps: {also[-1]['vs_f64']}")
        also.append(curved_bench(torch, lbm, case, args.storage, args.warmup, args.steps, main_run, pull_run))
        note(f"curved walls: {also[-1]['mlups']:.1f} MLUPS, pipe order {also[-1]['pipe_order']}")
        # SRT comparator: its step rate on the same run, and the stability sweep
        r = run_form(torch, lbm, dataclasses.replace(case, collision="srt2"), args.storage, args.warmup,
                     args.steps)
        also.append({"workload": f"{workload}_srt2", "storage": args.storage, "mlups": round(r["mlups"], 1),
                     "roofline_frac": roofline(r["n"], r["ms_per_step"], args.storage, None)["frac"],
                     "rate_vs_chm_mrt": round(r["mlups"] / main_run["mlups"], 3)})
        note(f"srt2: {also[-1]['mlups']:.1f} MLUPS")
        from paper_2101_11107_amd import stability
        sw = stability.sweep(128, 0, "f32")
        also.append({"workload": "stability_sweep_aneurysm128_steady_u0.06", "storage": "f32",
                     "steps": sw["rows"][0]["steps"], "lowest_stable_tau": sw["lowest_stable_tau"],
                     "rows": [{"tau": r["tau"], "fourier": r["fourier"],
                               "chm_mrt": r["chm_mrt"]["status"], "srt2": r["srt2"]["status"],
                               "srt2_failed_by_step": r["srt2"]["steps"] if r["srt2"]["status"] != "stable" else None}
                              for r in sw["rows"]]})
        note(f"stability: lowest stable tau {sw['lowest_stable_tau']}")
        from paper_2101_11107_amd import analysis
        rs = analysis.resolution_study(seed=48, n=256, cycles=4, storage="f32")
        also.append({"workload": "resolution_study_aneurysm256_vs_128", "storage": "f32", "cycles": 4,
                     "plane_similarity_index": {p["plane"]: round(p["similarity_index"], 5) for p in rs["planes"]},
                     "plane_points": {p["plane"]: p["points"] for p in rs["planes"]},
                     "si_histograms": {p["plane"]: p["si_histogram"] for p in rs["planes"]},
                     "probe_change_per_cycle_high": rs["periodicity_high"],
                     "probe_change_per_cycle_low": rs["periodicity_low"],
                     "seconds_high": rs["seconds_high"], "seconds_low": rs["seconds_low"],
                     "cost_ratio": rs["cost_ratio"]})
        note(f"resolution study: SI {also[-1]['plane_similarity_index']}, cost ratio {rs['cost_ratio']}")
        for st in ("f16s", "f32"):
            also.append(batch_bench(torch, lbm, 480, storage=st))
            note(f"batch {st}: {also[-1]['batched_mlups']:.1f} MLUPS batched, frac {also[-1]['roofline_frac']}")
        if not args.no_corrector:
            also.append(corrector_bench())
            note("corrector protocol done")
        line["also"] = also

    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(size, args.cpu_seconds)
        note(f"cpu baseline: {line['cpu_baseline']['value']} MLUPS")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
