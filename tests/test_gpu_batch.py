"""Batched stepping: every domain of a batch against the FP64 CPU oracle run
on that domain's own geometry and parameters (mixed relaxation times, both
batch modes), and bit-identical to stepping it alone in every execution
configuration the autotuner may pick."""

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
@pytest.mark.parametrize("mode", [0, 1])
def test_batch_matches_oracle(storage, tol, mode):
    """Four uneven geometries (boxes 64..128, tau between 0.51 and 1, each
    with its own Womersley inlet) stepped 100 times together by the batch
    kernels (mode 0: one launch per step for all domains; mode 1: one
    persistent launch), each against oracle O2 on its own case: the shifted
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
    assert cfg[0] in (0, 1) and cfg[1] in (128, 256, 512) and cfg[2] == 0 and cfg[4] >= 0
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
