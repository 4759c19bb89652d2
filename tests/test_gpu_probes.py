"""Monitoring points (a8 monitors: velocity at fixed points over time,
Sec. 2.2.2): the step kernel's probe records against lbm_moments and against
the FP64 oracle at the same times."""

import numpy as np
import pytest

import synth
from gpu_util import C

pytestmark = pytest.mark.gpu


def _probe_cells(case, k, seed):
    """k fluid cells, including ones next to walls and open boundaries."""
    fl = np.argwhere(case.mask == synth.FLUID)[:, ::-1]          # (x, y, z), x fastest
    rng = np.random.default_rng(seed)
    return fl[np.sort(rng.choice(len(fl), size=min(k, len(fl)), replace=False))].astype(np.int32)


def _moments_at(dom, cells):
    rho, u = dom.moments()
    xyz = dom.coords()
    idx = {tuple(p): i for i, p in enumerate(xyz.tolist())}
    sel = [idx[tuple(c)] for c in cells.tolist()]
    return np.concatenate([rho.cpu().numpy()[sel][:, None], u.cpu().numpy()[:, sel].T], axis=1)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-14), ("f32", 1e-6)])
def test_probe_records_equal_moments_at_those_times(storage, tol):
    from paper_2101_11107_amd import lbm
    print(f"case probes moments {storage}", flush=True)
    case = synth.random_tiny_case(1, nx=31, ny=9, nz=8)
    cells = _probe_cells(case, 12, 0)
    dom = lbm.Domain(case, storage=storage)
    dom.init()
    dom.set_probes(cells, every=5, capacity=10)
    dom.step(23)                                  # one graph of 16 steps and 7 single ones
    rec = dom.probe_records().cpu().numpy()
    dom.close()
    assert rec.shape == (4, len(cells), 4)
    ref = lbm.Domain(case, storage=storage)
    ref.init()
    for r in range(4):
        ref.step(5)
        m = _moments_at(ref, cells)
        assert np.max(np.abs(rec[r] - m)) < tol * max(1.0, np.max(np.abs(m)))
    ref.close()


def test_probe_records_match_the_oracle():
    from oracle import o2
    from paper_2101_11107_amd import lbm
    print("case probes oracle", flush=True)
    case = synth.aneurysm_case(64, 3)
    cells = _probe_cells(case, 3, 1)
    dom = lbm.Domain(case, storage="f64")
    dom.init()
    dom.set_probes(cells, every=40, capacity=3)
    dom.step(200)                                 # five record times, three kept
    rec = dom.probe_records().cpu().numpy()
    dom.close()
    assert rec.shape == (3, 3, 4)
    sim = o2.O2Sim(case, nthreads=8)
    nz, ny, nx = case.mask.shape
    k = [int(np.searchsorted((sim.coords[:, 2].astype(np.int64) * ny + sim.coords[:, 1]) * nx + sim.coords[:, 0],
                             (c[2] * ny + c[1]) * nx + c[0])) for c in cells.tolist()]
    for r in range(3):
        sim.run(40)
        rho, u = sim.macroscopic()
        ref = np.concatenate([rho[k][:, None], u[k]], axis=1)
        scale = max(np.max(np.abs(u)), 1e-300)
        assert np.max(np.abs(rec[r, :, 1:] - ref[:, 1:])) < 1e-12 * scale
        assert np.max(np.abs(rec[r, :, 0] - ref[:, 0])) < 1e-12


def test_probes_in_a_batch_equal_solo():
    from paper_2101_11107_amd import lbm
    print("case probes batch", flush=True)
    cases = [synth.aneurysm_case(64, 1), synth.random_tiny_case(3, nx=31, ny=9, nz=8)]
    cells = [_probe_cells(c, 5, 2) for c in cases]
    doms = [lbm.Domain(c, storage="f32") for c in cases]
    bufs = []
    for d, cl in zip(doms, cells):
        d.init()
        bufs.append(d.set_probes(cl, every=3, capacity=20))
    b = lbm.Batch(doms)
    b.step(37)
    got = [d.probe_records().cpu().numpy() for d in doms]
    b.close()
    for d in doms:
        d.close()
    for c, cl, g in zip(cases, cells, got):
        d = lbm.Domain(c, storage="f32")
        d.init()
        d.set_probes(cl, every=3, capacity=20)
        d.step(37)
        s = d.probe_records().cpu().numpy()
        d.close()
        assert g.shape == s.shape == (12, len(cl), 4)
        assert np.array_equal(g, s)
