"""Build the HIP library ``liblbm.so`` in-tree for gfx950 (MI355X)."""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblbm.so")
# (source, extra flags, object name): the step and batch kernels compile once
# per storage type, in parallel
SOURCES = [("lbm_kernels.hip", [], "lbm_kernels"), ("lbm_net.hip", [], "lbm_net"), ("lbm_net_noalloc.hip", [], "lbm_net_noalloc"),
           *[("lbm_step.hip", [f"-DLBM_STEP_STORAGE={k}"], f"lbm_step_{k}") for k in range(4)],
           *[("lbm_batch.hip", [f"-DLBM_BATCH_STORAGE={k}"], f"lbm_batch_{k}") for k in range(4)],
           ("lbm_api.cpp", [], "lbm_api"), ("lbm_batch_api.cpp", [], "lbm_batch_api"),
           ("lbm_net_api.cpp", [], "lbm_net_api")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # packed FP32 instructions stay off (hipcc warns that the host pass does not
    # know the feature; that warning is harmless)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiplies fuse into adds only within one source expression: with
    # fusion across statements, a product reused elsewhere in one variant of
    # a kernel (say, by the monitors) stays unfused there and fused in
    # another, and the variants would round differently
    "-ffp-contract=on",
]


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link liblbm.so."""
    import concurrent.futures
    import tempfile
    tmpdir = tempfile.mkdtemp(prefix="lbm_build_")
    objs = []
    cmds = []
    for src, extra, name in SOURCES:
        obj = os.path.join(tmpdir, name + ".o")
        objs.append(obj)
        cmds.append([HIPCC, *FLAGS, *extra, "-c", "-I", INCLUDE, "-I", CSRC, os.path.join(CSRC, src), "-o", obj])
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    for cmd, res in zip(cmds, results):
        if verbose:
            print(" ".join(cmd), flush=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed: " + cmd[-3])
    tmp = LIB + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("linking liblbm.so failed")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    os.rmdir(tmpdir)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
