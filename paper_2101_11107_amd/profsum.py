"""Summaries of rocprofv3 runs of the step kernel (text files under profiles/).

Input: the output folders of three rocprofv3 runs of the same bench command
(``--kernel-trace --stats``, ``--pmc FETCH_SIZE``, ``--pmc WRITE_SIZE``, CSV
output named ``run``), each starting with a plain device copy of known size
(``bench.py --copy-probe-mib``).  Output: the average duration of the step
kernel over its launches, and its HBM bytes per launch from the two
counters, each scaled by what the same counter reads for the copy (bytes the
copy moves / counter value).

    python -m paper_2101_11107_amd.profsum --dir <folder with trace/ fetch/ write/> \\
        --storage f32 --workload aneurysm512 --copy-mib 512 --cmd "<bench command>" --out <file>
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import re
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
POP_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
STEP = "k_step"           # demangled (k_step<...>) or mangled (...k_stepI...) names
COPY = "__amd_rocclr_copyBuffer"


def _code_only(text: str) -> str:
    """Source text without comments and with whitespace runs collapsed, so
    that editing a comment does not change the hash."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash() -> str:
    """Hash of the step kernel's code (comments and layout ignored); the
    bench accepts a summary only when it matches."""
    h = hashlib.sha256()
    for name in ("lbm_step.hip", "lbm_device.h", "lbm_internal.h"):
        with open(os.path.join(ROOT, "paper_2101_11107_amd", "csrc", name), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def _one(pattern: str) -> str:
    found = sorted(glob.glob(pattern, recursive=True))
    if not found:
        raise FileNotFoundError(pattern)
    return found[0]


def step_stats(trace_dir: str, last: int = 0) -> tuple:
    """(rows [(name, calls, avg us, min us, max us)], call-weighted average us
    of the step kernel, its launch count).  last > 0: only the last `last`
    step launches (per-dispatch trace), other kernels left out."""
    rows = []
    if last > 0:
        disp = []
        with open(_one(os.path.join(trace_dir, "**", "*kernel_trace.csv"))) as fh:
            for r in csv.DictReader(fh):
                if STEP in r["Kernel_Name"]:
                    disp.append((int(r["Dispatch_Id"]), r["Kernel_Name"],
                                 (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
        disp = sorted(disp)[-last:]
        by = {}
        for _, name, us in disp:
            by.setdefault(name, []).append(us)
        rows = [(n, len(v), sum(v) / len(v), min(v), max(v)) for n, v in by.items()]
    else:
        with open(_one(os.path.join(trace_dir, "**", "*kernel_stats.csv"))) as fh:
            for r in csv.DictReader(fh):
                rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                             float(r["MaxNs"]) / 1e3))
    steps = [r for r in rows if STEP in r[0]]
    calls = sum(r[1] for r in steps)
    avg = sum(r[1] * r[2] for r in steps) / calls
    return rows, avg, calls


def counter(run_dir: str, name: str, last: int = 0) -> tuple:
    """(copy value, [step values]) of one counter, per dispatch (KiB); last > 0:
    the last `last` step dispatches only."""
    copy = 0.0
    steps = []
    with open(_one(os.path.join(run_dir, "**", "*counter_collection.csv"))) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != name:
                continue
            v = float(r["Counter_Value"])
            if COPY in r["Kernel_Name"]:
                copy = max(copy, v)
            elif STEP in r["Kernel_Name"]:
                steps.append((int(r["Dispatch_Id"]), v))
    steps = [v for _, v in sorted(steps)]
    return copy, steps[-last:] if last > 0 else steps


def fluid_nodes(trace_dir: str) -> tuple:
    """(fluid nodes, curved wall links) from the bench result line captured
    beside the run."""
    with open(os.path.join(os.path.dirname(trace_dir.rstrip("/")), "trace.log")) as fh:
        for line in fh:
            if line.startswith("{"):
                cfg = json.loads(line)["config"]
                return int(cfg["fluid_nodes"]), int(cfg.get("wall_links", 0))
    raise ValueError("no bench result line in trace.log")


def summarize(folder: str, storage: str, workload: str, copy_mib: int, cmd: str, last: int = 0) -> str:
    trace, fetch, write = (os.path.join(folder, k) for k in ("trace", "fetch", "write"))
    rows, avg_us, calls = step_stats(trace, last)
    n, links = fluid_nodes(trace)
    moved_kib = copy_mib * 1024.0                     # the copy reads and writes this much
    fc, fs = counter(fetch, "FETCH_SIZE", last)
    wc, ws = counter(write, "WRITE_SIZE", last)
    f_scale, w_scale = moved_kib / fc, moved_kib / wc
    fetch_b = f_scale * sum(fs) / len(fs) * 1024.0
    write_b = w_scale * sum(ws) / len(ws) * 1024.0
    rec = 8 if storage == "f64" else 4
    alg = 54 * POP_BYTES[storage] * n + rec * links
    out = [f"# rocprofv3 summary: D3Q27 CHM-MRT step kernel (k_step), {storage} storage, workload {workload} "
           f"({n} fluid nodes{f', {links} curved wall links' if links else ''})",
           f"# kernel trace command : rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/trace -o run -- {cmd}",
           f"# FETCH_SIZE command   : rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/fetch -o run -- {cmd}",
           f"# WRITE_SIZE command   : rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/write -o run -- {cmd}",
           f"# summary command      : python -m paper_2101_11107_amd.profsum --dir <dir> --storage {storage} "
           f"--workload {workload} --copy-mib {copy_mib}{f' --last {last}' if last else ''} "
           f"--cmd \"<the bench command>\" --out <this file>",
           "#", "# kernel statistics (kernel-trace run" +
           (f"; the last {last} step launches, after the run's untimed spin-up steps)" if last else ")")]
    for name, c, a, lo, hi in sorted(rows, key=lambda r: -r[1] * r[2])[:8]:
        short = name.replace("(anonymous namespace)::", "").replace("(lbm::StepArgs)", "")
        out.append(f"#   {short[:78]:78s} calls {c:5d}  avg {a:9.3f} us  min {lo:9.3f}  max {hi:9.3f}")
    out += [f"#   step launches {calls}, call-weighted average duration {avg_us:.3f} us",
            "#",
            "# HBM traffic per step launch (two counter runs, each scaled by the same counter on a plain "
            f"{copy_mib} MiB device copy)",
            f"#   copy calibration: FETCH_SIZE {fc:.0f} KiB, WRITE_SIZE {wc:.0f} KiB for {moved_kib:.0f} KiB moved "
            f"-> scale {f_scale:.3f} / {w_scale:.3f}",
            f"#   step: FETCH_SIZE {sum(fs) / len(fs):.1f} KiB, WRITE_SIZE {sum(ws) / len(ws):.1f} KiB per dispatch "
            f"(n={len(fs)}, {len(ws)})",
            f"#   algorithmic bytes per launch (54 populations x {POP_BYTES[storage]} B x nodes"
            f"{f' + {rec} B weight x wall links' if links else ''}): {alg}",
            f"#   measured / algorithmic: read {fetch_b / (alg / 2):.3f}, write {write_b / (alg / 2):.3f}, "
            f"total {(fetch_b + write_b) / alg:.3f}",
            f"#   roofline: {alg / (avg_us * 1e-6) / 1e9:.1f} GB/s algorithmic on the kernel time "
            f"(frac {alg / (avg_us * 1e-6) / 8e12:.4f} of 8 TB/s)",
            f"kernel_source_sha256_16: {kernel_source_hash()}",
            f"avg_step_kernel_us: {avg_us:.4f}",
            f"fetch_bytes_per_launch: {fetch_b:.0f}",
            f"write_bytes_per_launch: {write_b:.0f}",
            f"hbm_bytes_per_launch: {fetch_b + write_b:.0f}",
            f"algorithmic_bytes_per_launch: {alg}"]
    return "\n".join(out) + "\n"


def _per_kernel(run_dir: str, patterns) -> dict:
    """{kernel name: {counter: [values per dispatch]}} of the kernels whose
    names contain one of the patterns, and the largest value per counter of
    the copy probe."""
    out, copy = {}, {}
    with open(_one(os.path.join(run_dir, "**", "*counter_collection.csv"))) as fh:
        for r in csv.DictReader(fh):
            name, c, v = r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"])
            if COPY in name:
                copy[c] = max(copy.get(c, 0.0), v)
            elif any(p in name for p in patterns):
                out.setdefault(name, {}).setdefault(c, []).append(v)
    return out, copy


def _short(name: str) -> str:
    return name.replace("(anonymous namespace)::", "").replace("lbmnet_dev::", "")[:70]


def summarize_kernels(folder: str, patterns, copy_mib: int, cmd: str, pmc_runs) -> str:
    """Per-kernel summary of a group of kernels (names containing one of the
    patterns): launches and average duration (trace run), HBM bytes per
    dispatch from FETCH_SIZE / WRITE_SIZE scaled by the copy probe, the
    bandwidth that gives, and the per-dispatch means of the counters of the
    extra runs pmc_runs = [(subfolder, command options)]."""
    rows, _, _ = step_stats_for(os.path.join(folder, "trace"), patterns)
    fetch, fcopy = _per_kernel(os.path.join(folder, "fetch"), patterns)
    write, wcopy = _per_kernel(os.path.join(folder, "write"), patterns)
    moved_kib = copy_mib * 1024.0
    fs, ws = moved_kib / fcopy["FETCH_SIZE"], moved_kib / wcopy["WRITE_SIZE"]
    extra = [(sub, _per_kernel(os.path.join(folder, sub), patterns)[0]) for sub, _ in pmc_runs]
    out = [f"# rocprofv3 summary of the kernels matching {list(patterns)}",
           f"# kernel trace command : rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/trace -o run -- {cmd}",
           f"# FETCH_SIZE command   : rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/fetch -o run -- {cmd}",
           f"# WRITE_SIZE command   : rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/write -o run -- {cmd}"]
    for sub, opts in pmc_runs:
        out.append(f"# {sub} command{' ' * max(1, 14 - len(sub))}: rocprofv3 {opts} --output-format csv -d <dir>/{sub} "
                   f"-o run -- {cmd}")
    out += [f"# copy calibration: FETCH_SIZE x {fs:.3f}, WRITE_SIZE x {ws:.3f} (a plain {copy_mib} MiB device copy)",
            "#", "# kernel                                                                 calls   avg us  "
            "read MB  write MB   GB/s   per-dispatch counter means"]
    for name, calls, avg, _, _ in sorted(rows, key=lambda r: -r[1] * r[2]):
        rd = fs * _mean(fetch.get(name, {}).get("FETCH_SIZE")) * 1024.0
        wr = ws * _mean(write.get(name, {}).get("WRITE_SIZE")) * 1024.0
        ctr = []
        for _, d in extra:
            for c, vals in sorted(d.get(name, {}).items()):
                ctr.append(f"{c} {_mean(vals):.4g}")
        out.append(f"#   {_short(name):70s} {calls:6d} {avg:8.2f} {rd / 1e6:8.2f} {wr / 1e6:9.2f} "
                   f"{(rd + wr) / (avg * 1e-6) / 1e9:7.1f}   {'; '.join(ctr)}")
    return "\n".join(out) + "\n"


def conv_gflop(coarse_voxels: int) -> tuple:
    """Useful convolution GFLOP of one network forward over coarse_voxels
    coarse voxels (2 x 27 x c_in x c_out per output voxel and layer, the
    half level holding 1/8 and the fine level 8 times the coarse voxels),
    and of one training step on it (forward, weight gradient, and input
    gradient of every layer but the first)."""
    from .net import layer_table
    scale = {0: 1.0, 1: 1.0 / 8.0, 2: 8.0}
    per = [2.0 * 27 * ci * co * coarse_voxels * scale[lev] / 1e9 for _, ci, co, _, lev, _ in layer_table()]
    return sum(per), 3.0 * sum(per) - per[0]


def conv_efficiency(trace_dir: str, train_steps: int, crop_voxels: int, forwards: int, grid_voxels: int) -> list:
    """Lines: convolution kernel time of the run, useful FLOPs, TFLOP/s and
    the fraction of the 2.5 PFLOP/s BF16 dense MFMA peak."""
    rows, _, _ = step_stats_for(trace_dir, ["k_conv"])
    secs = sum(c * a for _, c, a, _, _ in rows) * 1e-6
    _, train_g = conv_gflop(crop_voxels)
    fwd_g, _ = conv_gflop(grid_voxels)
    total = train_steps * train_g + forwards * fwd_g
    tf = total / 1e3 / secs
    return [f"# useful convolution flops: training step {train_g:.1f} GFLOP ({crop_voxels} coarse voxels), "
            f"full-grid forward {fwd_g:.1f} GFLOP ({grid_voxels} coarse voxels)",
            f"# {train_steps} training steps + {forwards} forwards: {total / 1e3:.2f} TFLOP in {secs * 1e3:.1f} ms of "
            f"convolution kernels -> {tf:.1f} TFLOP/s ({100 * tf / 2500:.2f} % of the 2.5 PFLOP/s BF16 dense peak)",
            f"conv_tflops_achieved: {tf:.2f}",
            f"conv_kernel_seconds: {secs:.4f}"]


def _mean(vals):
    return sum(vals) / len(vals) if vals else float("nan")


def step_stats_for(trace_dir: str, patterns) -> tuple:
    rows = []
    with open(_one(os.path.join(trace_dir, "**", "*kernel_stats.csv"))) as fh:
        for r in csv.DictReader(fh):
            if any(p in r["Name"] for p in patterns):
                rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                             float(r["MaxNs"]) / 1e3))
    return rows, None, None


def summarize_valu(runs, nodes: int, last: int, cmd: str) -> str:
    """Vector-instruction counts and VALU utilisation of the step kernel, per
    kernel variant, from one counter run per label (runs: [(label, dir)]).
    SQ_INSTS_VALU counts wavefront instructions; utilisation is
    SQ_ACTIVE_INST_VALU / 256 CUs / (GRBM_GUI_ACTIVE / 8 XCDs)."""
    waves = (nodes + 63) // 64
    out = [f"# rocprofv3 counter summary: D3Q27 CHM-MRT step kernel (k_step), workload aneurysm512 "
           f"({nodes} fluid nodes, {waves} wavefronts of 64 nodes)",
           f"# command: rocprofv3 --pmc SQ_INSTS_VALU SQ_ACTIVE_INST_VALU SQ_BUSY_CYCLES SQ_WAVE_CYCLES GRBM_GUI_ACTIVE "
           f"--output-format csv -d <dir>/<label> -o run -- {cmd}",
           f"# summary command: python -m paper_2101_11107_amd.profsum --valu-run <label>=<dir>/<label> ... "
           f"--nodes {nodes}{f' --last {last}' if last else ''} --cmd \"<the command>\" --out <this file>",
           "# per-dispatch means" + (f" over the last {last} step launches" if last else "") +
           "; GRBM_GUI_ACTIVE is summed over the 8 XCDs (one XCD's count is the kernel's cycles)",
           "# VALU utilisation = SQ_ACTIVE_INST_VALU / 256 CUs / (GRBM_GUI_ACTIVE / 8): issue cycles of one VALU "
           "instruction per CU cycle; kernel times under counter collection run a few per cent above the trace's"]
    for label, d in runs:
        disp = {}
        with open(_one(os.path.join(d, "**", "*counter_collection.csv"))) as fh:
            for r in csv.DictReader(fh):
                if STEP not in r["Kernel_Name"]:
                    continue
                e = disp.setdefault(int(r["Dispatch_Id"]), {"name": r["Kernel_Name"]})
                e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        ids = sorted(disp)[-last:] if last > 0 else sorted(disp)
        by = {}
        for k in ids:
            by.setdefault(disp[k]["name"], []).append(disp[k])
        for name, rows in sorted(by.items(), key=lambda kv: -len(kv[1])):
            mean = {c: sum(r.get(c, 0.0) for r in rows) / len(rows)
                    for c in ("SQ_INSTS_VALU", "SQ_ACTIVE_INST_VALU", "GRBM_GUI_ACTIVE")}
            cyc = mean["GRBM_GUI_ACTIVE"] / 8.0
            out.append(f"#   {label:12s} {_short(name).replace('void lbm::', '')[:58]:58s} dispatches {len(rows):4d}  "
                       f"-> {mean['SQ_INSTS_VALU'] / waves:6.0f} VALU instructions per wavefront, VALU utilisation "
                       f"{mean['SQ_ACTIVE_INST_VALU'] / 256.0 / cyc:.3f}, kernel {cyc / 2.4e3:.1f} us at 2.4 GHz")
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dir", default=None, help="the three runs of the step summary, or the kernel runs")
    ap.add_argument("--storage", choices=list(POP_BYTES))
    ap.add_argument("--workload")
    ap.add_argument("--kernels", default=None,
                    help="comma-separated name patterns: summarize those kernels instead of the step kernel")
    ap.add_argument("--pmc-run", action="append", default=[],
                    help="extra counter run as subfolder=rocprofv3 options (repeatable)")
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--last", type=int, default=0,
                    help="step kernel: average only the last N launches (the bench's warm-up and timed steps)")
    ap.add_argument("--conv-flops", default=None,
                    help="train_steps,crop_coarse_voxels,forwards,grid_coarse_voxels: add the convolution efficiency")
    ap.add_argument("--valu-run", action="append", default=[],
                    help="label=dir: VALU summary of the step kernel from that counter run (repeatable)")
    ap.add_argument("--nodes", type=int, default=0, help="fluid nodes (VALU summary)")
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.valu_run:
        text = summarize_valu([tuple(r.split("=", 1)) for r in a.valu_run], a.nodes, a.last, a.cmd)
    elif a.kernels:
        runs = [tuple(r.split("=", 1)) for r in a.pmc_run]
        text = summarize_kernels(a.dir, a.kernels.split(","), a.copy_mib, a.cmd, runs)
        if a.conv_flops:
            ts, cv, fw, gv = (int(v) for v in a.conv_flops.split(","))
            text += "\n".join(conv_efficiency(os.path.join(a.dir, "trace"), ts, cv, fw, gv)) + "\n"
    else:
        text = summarize(a.dir, a.storage, a.workload, a.copy_mib, a.cmd, a.last)
    with open(a.out, "w") as fh:
        fh.write(text)
    print(text, end="")


if __name__ == "__main__":
    main()
