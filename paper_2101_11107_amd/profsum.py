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
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
POP_BYTES = {"f64": 8, "f32": 4, "f16s": 2, "bf16s": 2}
STEP = "k_step"           # demangled (k_step<...>) or mangled (...k_stepI...) names
COPY = "__amd_rocclr_copyBuffer"


def kernel_source_hash() -> str:
    """Hash of the step kernel's sources (the bench accepts a summary only
    when it matches)."""
    h = hashlib.sha256()
    for name in ("lbm_kernels.hip", "lbm_device.h", "lbm_internal.h"):
        with open(os.path.join(ROOT, "paper_2101_11107_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _one(pattern: str) -> str:
    found = sorted(glob.glob(pattern, recursive=True))
    if not found:
        raise FileNotFoundError(pattern)
    return found[0]


def step_stats(trace_dir: str) -> tuple:
    """(rows [(name, calls, avg us, min us, max us)], call-weighted average us
    of the step kernel, its launch count)."""
    rows = []
    with open(_one(os.path.join(trace_dir, "**", "*kernel_stats.csv"))) as fh:
        for r in csv.DictReader(fh):
            rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                         float(r["MaxNs"]) / 1e3))
    steps = [r for r in rows if STEP in r[0]]
    calls = sum(r[1] for r in steps)
    avg = sum(r[1] * r[2] for r in steps) / calls
    return rows, avg, calls


def counter(run_dir: str, name: str) -> tuple:
    """(copy value, [step values]) of one counter, per dispatch (KiB)."""
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
                steps.append(v)
    return copy, steps


def fluid_nodes(trace_dir: str) -> int:
    """Fluid-node count from the bench result line captured beside the run."""
    with open(os.path.join(os.path.dirname(trace_dir.rstrip("/")), "trace.log")) as fh:
        for line in fh:
            if line.startswith("{"):
                return int(json.loads(line)["config"]["fluid_nodes"])
    raise ValueError("no bench result line in trace.log")


def summarize(folder: str, storage: str, workload: str, copy_mib: int, cmd: str) -> str:
    trace, fetch, write = (os.path.join(folder, k) for k in ("trace", "fetch", "write"))
    rows, avg_us, calls = step_stats(trace)
    n = fluid_nodes(trace)
    moved_kib = copy_mib * 1024.0                     # the copy reads and writes this much
    fc, fs = counter(fetch, "FETCH_SIZE")
    wc, ws = counter(write, "WRITE_SIZE")
    f_scale, w_scale = moved_kib / fc, moved_kib / wc
    fetch_b = f_scale * sum(fs) / len(fs) * 1024.0
    write_b = w_scale * sum(ws) / len(ws) * 1024.0
    alg = 54 * POP_BYTES[storage] * n
    out = [f"# rocprofv3 summary: D3Q27 CHM-MRT step kernel (k_step), {storage} storage, workload {workload} "
           f"({n} fluid nodes)",
           f"# kernel trace command : rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/trace -o run -- {cmd}",
           f"# FETCH_SIZE command   : rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/fetch -o run -- {cmd}",
           f"# WRITE_SIZE command   : rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/write -o run -- {cmd}",
           f"# summary command      : python -m paper_2101_11107_amd.profsum --dir <dir> --storage {storage} "
           f"--workload {workload} --copy-mib {copy_mib} --cmd \"<the bench command>\" --out <this file>",
           "#", "# kernel statistics (kernel-trace run)"]
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
            f"#   algorithmic bytes per launch (54 populations x {POP_BYTES[storage]} B x nodes): {alg}",
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--dir", required=True)
    ap.add_argument("--storage", required=True, choices=list(POP_BYTES))
    ap.add_argument("--workload", required=True)
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    text = summarize(a.dir, a.storage, a.workload, a.copy_mib, a.cmd)
    with open(a.out, "w") as fh:
        fh.write(text)
    print(text, end="")


if __name__ == "__main__":
    main()
