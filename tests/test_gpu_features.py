"""GPU tests of invariants, monitors, checkpointing, averaging and failure handling."""

import numpy as np
import pytest

import synth
from gpu_util import C, W, gpu_run, oracle_order, oracle_post

pytestmark = pytest.mark.gpu


def _closed(case):
    case.mask[case.mask >= 2] = synth.SOLID
    case.inlet = None
    case.g = (0.0, 0.0, 0.0)
    return case


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
def test_rest_state_is_bitwise_fixed_point(storage):
    """Shifted storage makes the rest state exactly zero; collision, bounce-back
    and streaming keep it exactly zero in every storage type."""
    print(f"case rest aneurysm128 {storage}", flush=True)
    case = _closed(synth.aneurysm_case(128, seed=3))
    dom, f = gpu_run(case, storage, 37)
    dom.close()
    assert np.count_nonzero(f) == 0


def test_determinism_bitwise():
    print("case determinism aneurysm256 f32", flush=True)
    case = synth.aneurysm_case(256, seed=0)
    d1, f1 = gpu_run(case, "f32", 50)
    m1 = d1.monitors()
    d1.close()
    d2, f2 = gpu_run(case, "f32", 50)
    m2 = d2.monitors()
    d2.close()
    assert np.array_equal(f1, f2)
    assert np.array_equal(m1, m2)


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_checkpoint_resume_bitwise(storage):
    """N + M steps equal N steps, checkpoint, restore into a fresh domain, M steps."""
    from paper_2101_11107_amd import lbm
    print(f"case checkpoint aneurysm256 {storage}", flush=True)
    case = synth.aneurysm_case(256, seed=1)
    a = lbm.Domain(case, storage=storage)
    a.init()
    a.step(37 + 29)
    fa = a.populations().cpu().numpy()
    a.close()
    b = lbm.Domain(case, storage=storage)
    b.init()
    b.step(37)
    blob = b.get_state()
    b.close()
    c = lbm.Domain(case, storage=storage)
    c.set_state(blob)
    assert c.time() == 37
    c.step(29)
    fc = c.populations().cpu().numpy()
    c.close()
    assert np.array_equal(fa, fc)


def test_checkpoint_header_is_validated():
    from paper_2101_11107_amd import lbm
    case = synth.aneurysm_case(128, seed=0)
    a = lbm.Domain(case, storage="f32")
    a.init()
    a.step(3)
    blob = bytearray(a.get_state())
    blob[0] ^= 0xFF
    with pytest.raises(lbm.LbmError) as e:
        a.set_state(bytes(blob))
    assert e.value.code == lbm.LBM_EINVAL
    other = lbm.Domain(case, storage="f16s")
    with pytest.raises(lbm.LbmError):
        other.set_state(a.get_state())
    # another node order (row-tile edge) or another layout version is refused
    reordered = lbm.Domain(case, storage="f32", row_tile=4)
    with pytest.raises(lbm.LbmError):
        reordered.set_state(a.get_state())
    old = bytearray(a.get_state())
    old[8:12] = (1).to_bytes(4, "little")
    with pytest.raises(lbm.LbmError):
        a.set_state(bytes(old))
    a.close()
    other.close()
    reordered.close()


def test_mass_balance_every_step_open_system():
    """M(t+1) - M(t) = inlet flux + outlet flux, step by step (FP64 storage)."""
    from paper_2101_11107_amd import lbm
    print("case mass balance aneurysm256 f64", flush=True)
    case = synth.aneurysm_case(256, seed=0)
    dom = lbm.Domain(case, storage="f64")
    dom.init()
    dom.step(1)
    prev = dom.monitors()
    for _ in range(12):
        dom.step(1)
        m = dom.monitors()
        assert abs((m[0] - prev[0]) - (m[7] + m[8])) < 1e-12 * m[0]
        prev = m
    dom.close()


@pytest.mark.parametrize("seed", [0, 2])
def test_monitors_match_oracle(seed):
    """Mass, momentum, wall force and boundary fluxes of the last step (FP64)."""
    print(f"case monitors tiny{seed}", flush=True)
    case = synth.random_tiny_case(seed, nx=11, ny=9, nz=8)
    dom, _ = gpu_run(case, "f64", 20)
    mon = dom.monitors()
    dom.close()
    from oracle import o2
    sim = o2.O2Sim(case, nthreads=4)
    ref = sim.run(20)
    scale = np.maximum(np.abs(ref), 1.0)
    assert np.max(np.abs(mon - ref) / scale) < 1e-12


def test_pipe_monitors_f32_mass_drift():
    """Closed pipe in FP32 storage: mass drift stays at FP32 rounding level."""
    print("case pipe f32 mass", flush=True)
    case = synth.pipe_case()
    dom, _ = gpu_run(case, "f32", 2000)
    mon = dom.monitors()
    dom.close()
    assert abs(mon[0] - 20224.0) / 20224.0 < 1e-7
    # wall force balances the body force in the developed flow: F = M g
    assert abs(mon[4] - 20224.0 * 1e-6) < 0.05 * 20224.0 * 1e-6


def test_time_average_matches_mean_of_moments():
    import torch
    from paper_2101_11107_amd import lbm
    case = synth.aneurysm_case(128, seed=0)
    dom = lbm.Domain(case, storage="f32")
    dom.init()
    dom.step(5)
    dom.average(lbm.LBM_AVG_RESET)
    acc = None
    for _ in range(6):
        dom.step(3)
        dom.average(lbm.LBM_AVG_ACCUMULATE)
        _, u = dom.moments()
        acc = u.clone() if acc is None else acc + u
    avg = dom.average(lbm.LBM_AVG_READ)
    torch.cuda.synchronize()
    ref = (acc / 6).cpu().numpy()
    assert np.max(np.abs(avg.cpu().numpy() - ref)) < 1e-15
    dom.close()


def test_nonfinite_state_reported_unstable():
    """A NaN restored into the state is reported by the monitor watchdog."""
    import struct
    from paper_2101_11107_amd import lbm
    case = synth.aneurysm_case(128, seed=0)
    dom = lbm.Domain(case, storage="f32")
    dom.init()
    dom.step(2)
    blob = bytearray(dom.get_state())
    # header of the state blob: magic, version, storage, n, nspec, npad, t,
    # population bytes, row-tile edge, population tile
    hdr = 8 + 4 + 4 + 8 * 4 + 8 + 4 + 4
    blob[hdr: hdr + 4] = struct.pack("<f", float("nan"))
    dom.set_state(bytes(blob))
    dom.step(2)
    with pytest.raises(lbm.LbmError) as e:
        dom.monitors()
    assert e.value.code == lbm.LBM_EUNSTABLE
    dom.close()


def test_step_before_init_is_rejected():
    from paper_2101_11107_amd import lbm
    case = synth.aneurysm_case(128, seed=0)
    dom = lbm.Domain(case, storage="f32")
    with pytest.raises(lbm.LbmError) as e:
        dom.step(1)
    assert e.value.code == lbm.LBM_ESTATE
    with pytest.raises(lbm.LbmError):
        dom.monitors()
    dom.close()


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_tracked_average_matches_separate_accumulation(storage, tol):
    """Averaging inside the step kernel (LBM_AVG_TRACK, graphs allowed) equals
    adding the moments after every single step (LBM_AVG_ACCUMULATE): the same
    velocities, computed in the collision's precision instead of FP64."""
    from paper_2101_11107_amd import lbm
    print(f"case tracked average aneurysm128 {storage}", flush=True)
    case = synth.aneurysm_case(128, seed=5)
    steps = 67
    a = lbm.Domain(case, storage=storage)
    a.init()
    a.average(lbm.LBM_AVG_RESET)
    for _ in range(steps):
        a.step(1)
        a.average(lbm.LBM_AVG_ACCUMULATE)
    ua = a.average(lbm.LBM_AVG_READ).cpu().numpy()
    fa = a.populations().cpu().numpy()
    a.close()
    b = lbm.Domain(case, storage=storage)
    b.init()
    b.average(lbm.LBM_AVG_RESET)
    b.average(lbm.LBM_AVG_TRACK)
    b.step(steps)
    ub = b.average(lbm.LBM_AVG_READ).cpu().numpy()
    fb = b.populations().cpu().numpy()
    b.close()
    assert np.array_equal(fa, fb)          # tracking does not change the run
    assert np.max(np.abs(ua - ub)) <= tol * np.max(np.abs(ua))


def test_tracked_average_through_batch_equals_solo():
    from paper_2101_11107_amd import lbm
    print("case tracked average batch f16s", flush=True)
    cases = [synth.aneurysm_case(64, seed=s) for s in (1, 2)]
    doms = [lbm.Domain(c, storage="f16s") for c in cases]
    for d in doms:
        d.init()
    b = lbm.Batch(doms)
    b.step(8)                                  # tables built without tracking
    for d in doms:
        d.average(lbm.LBM_AVG_RESET)
        d.average(lbm.LBM_AVG_TRACK)
    b.step(40)                                 # the batch sees the tracking change
    got = [d.average(lbm.LBM_AVG_READ).cpu().numpy() for d in doms]
    b.close()
    for d in doms:
        d.close()
    # the batch run is 8 steps ahead of the solo runs: compare with solo runs of 48
    ref = []
    for c in cases:
        d = lbm.Domain(c, storage="f16s")
        d.init()
        d.step(8)
        d.average(lbm.LBM_AVG_TRACK)
        d.step(40)
        ref.append(d.average(lbm.LBM_AVG_READ).cpu().numpy())
        d.close()
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)


def test_resolution_study_runs_and_is_consistent():
    """The resolution study on a small geometry (128^3 against 64^3, two
    periods): three planes with a similarity index in (0, 1], probe changes
    for the second period, and a coarse run cheaper than the fine one."""
    from paper_2101_11107_amd import analysis
    print("case resolution study 128/64", flush=True)
    res = analysis.resolution_study(seed=3, n=128, cycles=2)
    assert len(res["planes"]) == 3
    for p in res["planes"]:
        assert p["points"] > 0 and 0.0 < p["similarity_index"] <= 1.0
        assert abs(sum(p["si_histogram"]) - 1.0) < 1e-4     # entries rounded to 5 decimals
    assert len(res["periodicity_high"]) == 1 and len(res["periodicity_low"]) == 1
    assert res["fluid_nodes_high"] > 6 * res["fluid_nodes_low"]


@pytest.mark.parametrize("tau", [0.6, 1.5])
def test_wall_position_fixed_by_the_third_order_rate(tau):
    """The oracle's pin P12 on the GPU (the general-rate CHM-MRT kernel, FP64):
    with (1/s2 - 1/2)(1/s3 - 1/2) = 3/16 the steady channel profile with
    halfway walls is exact to rounding."""
    import dataclasses
    from paper_2101_11107_amd import lbm
    print(f"case channel wall position tau {tau}", flush=True)
    H, g = 8, 1e-6
    s3 = 1.0 / (0.5 + 0.1875 / (tau - 0.5))
    case = dataclasses.replace(synth.channel_case(4, H + 2, 2, tau, g), rates=(s3, 1.0, 1.0, 1.0))
    dom = lbm.Domain(case, storage="f64")
    dom.init()
    dom.step(int(40 * H * H / case.nu))
    _, u = dom.moments()
    y = dom.coords()[:, 1].astype(float)
    dom.close()
    ua = g / (2 * case.nu) * (y - 0.5) * (H + 0.5 - y)
    assert np.abs(u.cpu().numpy()[0] - ua).max() / ua.max() < 1e-9
