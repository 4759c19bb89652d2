"""Host-side pieces of the benchmark: the roofline arithmetic, the profile
reader (only summaries taken on the current kernel source count) and the
refusal of multi-GPU runs."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_roofline_uses_algorithmic_bytes():
    import bench
    r = bench.roofline(1000, 0.001, "f32", None)     # 1000 nodes in 1 us
    assert r["algorithmic_bytes_per_launch"] == 54 * 4 * 1000
    assert abs(r["achieved"] - 216.0) < 1e-9           # 216 kB per us = 216 GB/s
    assert r["peak"] == 8000.0 and r["unit"] == "GB/s" and r["bound"] == "hbm"
    assert abs(r["frac"] - 0.027) < 1e-12
    assert bench.roofline(10, 1.0, "f16s", None)["algorithmic_bytes_per_launch"] == 54 * 2 * 10
    # curved walls add one weight per wall link (8 B with FP64 storage, 4 B otherwise)
    assert bench.roofline(10, 1.0, "f16s", None, 7)["algorithmic_bytes_per_launch"] == 54 * 2 * 10 + 4 * 7
    assert bench.roofline(10, 1.0, "f64", None, 7)["algorithmic_bytes_per_launch"] == 54 * 8 * 10 + 8 * 7


def test_committed_profiles_match_current_kernel_source():
    import bench
    for st, wl in (("f32", "aneurysm512"), ("f32", "aneurysm256"), ("f16s", "aneurysm512"), ("f64", "aneurysm512"),
                   ("bf16s", "aneurysm512"), ("f32", "aneurysm512_curved")):
        prof = bench.read_profile(st, wl)
        assert prof, f"profiles/traffic_k_step_{st}_{wl}.txt is missing or was taken on another kernel source"
        alg = 54 * bench.POP_BYTES[st] * (262221 if wl == "aneurysm256" else 2121645)
        if wl.endswith("_curved"):
            alg += 4 * 1457610          # FP32 weight per wall link of the 512^3 geometry
        assert int(prof["algorithmic_bytes_per_launch"]) == alg
        assert 1.0 <= float(prof["hbm_bytes_per_launch"]) / alg < 1.3
        assert float(prof["avg_step_kernel_us"]) > 0


def test_multi_gpu_request_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode != 0
    assert "one GPU" in res.stderr
