"""Batched stepping: every domain of a batch against the FP64 CPU oracle run
on that domain's own geometry and parameters (mixed relaxation times, the
three batch modes), and bit-identical to stepping it alone in every execution
configuration the autotuner may pick, including in-place streaming."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _small_batch(storage, n=6):
    cases = synth.batch_cases(first_seed=2000, count=n)
    return [c for c in cases if c.mask.shape[0] <= 128][:4] + cases[:2]


def _solo(case, storage, steps):
    from paper_2101_11107_amd import lbm
    d = lbm.Domain(case, storage=storage)
    d.init()
    d.step(steps)
    f = d.populations().cpu().numpy()
    m = d.monitors()
    d.close()
    return f, m


@pytest.mark.parametrize("storage", ["f16s", "f32"])
@pytest.mark.parametrize("cfg", [(0, 128, 0, 0, 0), (0, 256, 1, 0, 1), (0, 512, 0, 0, 0), (1, 256, 0, 0, 1),
                                 (1, 512, 1, 0, 0), (1, 128, 0, 64, 2)])
def test_batch_equals_solo_bitwise(storage, cfg):
    from paper_2101_11107_amd import lbm
    if storage.startswith(("f16", "bf16")) and cfg[2]:
        cfg = (cfg[0], cfg[1], 0, cfg[3], cfg[4])
    print(f"case batch {storage} cfg {cfg}", flush=True)
    cases = _small_batch(storage)
    steps = 37                       # two graph replays and five single launches
    doms = [lbm.Domain(c, storage=storage) for c in cases]
    for d in doms:
        d.init()
    b = lbm.Batch(doms)
    b.set_config(cfg)
    b.step(steps)
    b.status()
    got = []
    for d in doms:
        got.append((d.populations().cpu().numpy(), d.monitors(), d.time()))
    b.close()
    for d in doms:
        d.close()
    for c, (f, m, t) in zip(cases, got):
        fs, ms = _solo(c, storage, steps)
        assert t == steps
        assert np.array_equal(f, fs)
        # monitor sums may differ in order (different work-group sizes)
        assert np.max(np.abs(m - ms) / np.maximum(np.abs(ms), 1.0)) < 1e-12


_ORACLE = {}   # oracle results per case, shared by the parametrizations


@pytest.mark.parametrize("storage,tol", [("f32", 1e-5), ("f16s", 1e-3)])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_batch_matches_oracle(storage, tol, mode):
    """Four uneven geometries (boxes 64..128, tau between 0.51 and 1, each
    with its own Womersley inlet) stepped 100 times together by the batch
    kernels (mode 0: one launch per step for all domains; mode 1: one
    persistent launch; mode 2: one launch per step, streamed in place, read
    back through the pull layout), each against oracle O2 on its own case: the shifted
    post-collision populations element by element and the velocity error,
    within the storage form's bound (FP32 1e-5, f16s 1e-3 of the largest
    value)."""
    from gpu_util import eps_u, moments_from_post, oracle_order, oracle_post
    from paper_2101_11107_amd import lbm
    cases = [c for c in synth.batch_cases(first_seed=2000, count=12) if c.mask.shape[0] <= 128][:4]
    assert len(cases) == 4 and len({round(c.tau, 6) for c in cases}) == 4
    print(f"case batch vs oracle {storage} mode {mode}: {[c.name for c in cases]}", flush=True)
    steps = 100
    doms = [lbm.Domain(c, storage=storage) for c in cases]
    for d in doms:
        d.init()
    b = lbm.Batch(doms)
    b.set_config((mode, 256, 0, 0, 0))
    b.step(steps)
    b.status()
    got = []
    for c, d in zip(cases, doms):
        f = d.populations().cpu().numpy().T
        got.append(f[oracle_order(d.coords(), c.mask)])
    b.close()
    for d in doms:
        d.close()
    for c, f in zip(cases, got):
        if c.name not in _ORACLE:
            _, ref, _, u_ref = oracle_post(c, steps)
            _ORACLE[c.name] = (ref, u_ref)
        ref, u_ref = _ORACLE[c.name]
        err = float(np.max(np.abs(f - ref)) / np.max(np.abs(ref)))
        _, u = moments_from_post(f, c.g)
        print(f"  {c.name}: tau {c.tau:.4f}  population error {err:.2e}  eps_u {eps_u(u, u_ref):.2e}", flush=True)
        assert err < tol
        assert eps_u(u, u_ref) < tol


def test_batch_autotune_and_continue():
    """The autotuner picks a valid configuration; stepping continues from the
    advanced state and matches solo runs of the same total length."""
    from paper_2101_11107_amd import lbm
    print("case batch autotune f16s", flush=True)
    cases = _small_batch("f16s")
    doms = [lbm.Domain(c, storage="f16s") for c in cases]
    for d in doms:
        d.init()
    b = lbm.Batch(doms)
    best = b.autotune(trial_steps=16, want_time=True)
    assert best > 0
    cfg = b.config()
    assert cfg[0] in (0, 1, 2) and cfg[1] in (128, 256, 512) and cfg[2] == 0 and cfg[4] >= 0
    assert cfg[0] != 2 or cfg[1] == 256
    t0 = doms[0].time()
    b.step(20)
    b.status()
    f0 = doms[0].populations().cpu().numpy()
    total = doms[0].time()
    assert total == t0 + 20
    b.close()
    for d in doms:
        d.close()
    fs, _ = _solo(cases[0], "f16s", total)
    assert np.array_equal(f0, fs)


def test_batch_rejects_mixed_storage():
    from paper_2101_11107_amd import lbm
    cases = _small_batch("f16s", n=2)
    a = lbm.Domain(cases[0], storage="f16s")
    c = lbm.Domain(cases[1], storage="f32")
    with pytest.raises(lbm.LbmError) as e:
        lbm.Batch([a, c])
    assert e.value.code == lbm.LBM_EINVAL
    a.close()
    c.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("group_mb", [0, 1])
def test_inplace_batch_equals_solo_bitwise(storage, group_mb):
    """Mode 2 (in place): 37 steps (an odd count ends in the streamed layout),
    a read of one domain's state (which brings that domain back to the pull
    layout, so the next call realigns every domain), 20 more steps, 5 with
    pull launches and 3 in place again; each domain bit-identical to 65 steps
    of its own stepping, in one group or in several."""
    from paper_2101_11107_amd import lbm
    print(f"case inplace batch {storage} group {group_mb}", flush=True)
    cases = _small_batch(storage)
    doms = [lbm.Domain(c, storage=storage) for c in cases]
    for d in doms:
        d.init()
    b = lbm.Batch(doms)
    cfg = (2, 256, 0, 0, group_mb)
    b.set_config(cfg)
    b.step(37)
    b.status()
    mid = doms[1].populations().cpu().numpy()
    b.step(20)
    b.set_config((0, 256, 0, 0, group_mb))
    b.step(5)
    b.set_config(cfg)
    b.step(3)
    b.status()
    got = [(d.populations().cpu().numpy(), d.monitors(), d.time()) for d in doms]
    b.close()
    for d in doms:
        d.close()
    assert np.array_equal(mid, _solo(cases[1], storage, 37)[0])
    for c, (f, m, t) in zip(cases, got):
        fs, ms = _solo(c, storage, 65)
        assert t == 65
        assert np.array_equal(f, fs)
        assert np.max(np.abs(m - ms) / np.maximum(np.abs(ms), 1.0)) < 1e-12


def test_inplace_batch_mixed_forms_probes_average():
    """Mode 2 over CHM-MRT (rates one and general rates) and SRT domains, with
    monitoring points on one and in-kernel velocity averaging on another:
    populations, probe records and averages bit-identical to solo runs."""
    import dataclasses
    from test_gpu_probes import _probe_cells
    from paper_2101_11107_amd import lbm
    print("case inplace batch mixed forms, probes, averages", flush=True)
    cases = [synth.aneurysm_case(64, 1), dataclasses.replace(synth.aneurysm_case(64, 2), collision="srt2"),
             synth.random_tiny_case(1, nx=31, ny=9, nz=8), synth.random_tiny_case(3, nx=31, ny=9, nz=8)]
    cells = _probe_cells(cases[0], 5, 2)
    steps = 37

    def setup(d, k):
        d.init()
        if k == 0:
            d.set_probes(cells, every=3, capacity=20)
        if k == 2:
            d.average(lbm.LBM_AVG_RESET)
            d.average(lbm.LBM_AVG_TRACK)

    def read(d, k):
        f = d.populations().cpu().numpy()
        extra = d.probe_records().cpu().numpy() if k == 0 else (
            d.average(lbm.LBM_AVG_READ).cpu().numpy() if k == 2 else None)
        return f, extra

    doms = [lbm.Domain(c, storage="f32") for c in cases]
    for k, d in enumerate(doms):
        setup(d, k)
    b = lbm.Batch(doms)
    b.set_config((2, 256, 0, 0, 0))
    b.step(steps)
    b.status()
    got = [read(d, k) for k, d in enumerate(doms)]
    b.close()
    for d in doms:
        d.close()
    for k, (c, (fb, eb)) in enumerate(zip(cases, got)):
        d = lbm.Domain(c, storage="f32")
        setup(d, k)
        d.step(steps)
        fs, es = read(d, k)
        d.close()
        assert np.array_equal(fb, fs)
        if eb is not None:
            assert np.array_equal(eb, es)


def test_inplace_batch_rejections():
    """Mode 2 takes 256 threads and cached stores only, and no curved walls."""
    from paper_2101_11107_amd import lbm
    print("case inplace batch rejections", flush=True)
    cases = _small_batch("f32", n=2)[:2]
    doms = [lbm.Domain(c, storage="f32") for c in cases]
    for d in doms:
        d.init()
    b = lbm.Batch(doms)
    for cfg in [(2, 128, 0, 0, 0), (2, 512, 0, 0, 0), (2, 256, 1, 0, 0), (3, 256, 0, 0, 0)]:
        with pytest.raises(lbm.LbmError) as e:
            b.set_config(cfg)
        assert e.value.code == lbm.LBM_EINVAL
    b.close()
    for d in doms:
        d.close()
    # a batch with a curved-wall domain: the configuration is valid, the step
    # is refused and the state is left as it was
    case = synth.aneurysm_case(64, 1)
    links = synth.wall_links(case.mask, 0)
    doms = [lbm.Domain(cases[0], storage="f32"),
            lbm.Domain(case, storage="f32", wall_q=(links, synth.wall_distances(case, links)))]
    for d in doms:
        d.init()
    b = lbm.Batch(doms)
    b.set_config((2, 256, 0, 0, 0))
    with pytest.raises(lbm.LbmError) as e:
        b.step(3)
    assert e.value.code == lbm.LBM_EINVAL
    assert [d.time() for d in doms] == [0, 0]
    b.set_config((0, 256, 0, 0, 0))
    b.step(3)
    b.status()
    assert [d.time() for d in doms] == [3, 3]
    b.close()
    for d in doms:
        d.close()
