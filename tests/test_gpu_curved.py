"""Curved walls on the GPU (Sec. 2.1.4, Eq. (9)-(10)): interpolated bounce-back
through the C ABI against the FP64 oracle with the same wall distances.

Bars as for the rest of the step: FP64 storage within 1e-13 on populations
(1e-12 relative on velocities), FP32 within 1e-5 relative.
"""

import math

import numpy as np
import pytest

import synth
from gpu_util import eps_u, gpu_run, moments_from_post, oracle_post

pytestmark = pytest.mark.gpu


def _random_q(case, seed):
    links = synth.wall_links(case.mask, case.periodic)
    return links, synth.random_wall_distances(links, seed)


@pytest.mark.parametrize("seed", [0, 1, 3, 5])
def test_random_wall_distances_f64_population_parity(seed):
    """Tiny random masks with every cell type and periodic axes; every wall
    link gets a random q in [0.02, 1]: both branches of Eq. (9), the halfway
    fallback where the node behind is not fluid, and nodes that also carry
    open links."""
    print(f"case curved tiny{seed} f64", flush=True)
    case = synth.random_tiny_case(seed, nx=11, ny=9, nz=8)
    wq = _random_q(case, seed)
    dom, f = gpu_run(case, "f64", 20, wall_q=wq)
    mon = dom.monitors()
    dom.close()
    sim, ref, _, _ = oracle_post(case, 20, wall_q=wq)
    assert np.max(np.abs(f - ref)) < 1e-13
    # the monitors of the last step: mass, momentum, wall force, boundary fluxes
    from oracle import o2
    s2 = o2.O2Sim(case, nthreads=4, wall_q={tuple(int(v) for v in lk): float(q) for lk, q in zip(*wq)})
    mref = s2.run(20)
    assert np.max(np.abs(mon - mref) / np.maximum(np.abs(mref), 1.0)) < 1e-12


@pytest.mark.parametrize("seed", [0, 3])
def test_random_wall_distances_f32_population_parity(seed):
    print(f"case curved tiny{seed} f32", flush=True)
    case = synth.random_tiny_case(seed, nx=11, ny=9, nz=8)
    wq = _random_q(case, seed + 100)
    dom, f = gpu_run(case, "f32", 20, wall_q=wq)
    dom.close()
    _, ref, _, _ = oracle_post(case, 20, wall_q=wq)
    assert np.max(np.abs(f - ref)) < 1e-5 * np.max(np.abs(ref))


@pytest.mark.parametrize("storage,tol", [("f16s", 1e-3), ("bf16s", 8e-3)])
@pytest.mark.parametrize("seed", [0, 3])
def test_random_wall_distances_reduced_storage(storage, tol, seed):
    """The 2-byte storage forms blend in FP32 with FP32 weights and round the
    result once on store: populations within the form's bound (1e-3 f16s,
    8e-3 bf16s, of the largest population) after 20 steps."""
    print(f"case curved tiny{seed} {storage}", flush=True)
    case = synth.random_tiny_case(seed, nx=11, ny=9, nz=8)
    wq = _random_q(case, seed)
    dom, f = gpu_run(case, storage, 20, wall_q=wq)
    dom.close()
    _, ref, _, _ = oracle_post(case, 20, wall_q=wq)
    assert np.max(np.abs(f - ref)) < tol * np.max(np.abs(ref))


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_half_distance_equals_halfway_bounce_back_bitwise(storage):
    """q = 1/2 on every wall link through the curved-wall path gives the
    populations of the plain halfway bounce-back domain bit for bit."""
    print(f"case curved half {storage}", flush=True)
    case = synth.random_tiny_case(2, nx=31, ny=9, nz=8)
    links = synth.wall_links(case.mask, case.periodic)
    d1, f1 = gpu_run(case, storage, 25)
    d1.close()
    d2, f2 = gpu_run(case, storage, 25, wall_q=(links, np.full(len(links), 0.5)))
    d2.close()
    assert np.array_equal(f1, f2)


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_pipe_exact_wall_distances(storage, tol):
    """Pipe off the lattice axis with the exact circular-wall distances, at
    the config-1 force g = 1e-6 (u_max 2.5e-4): velocities after 2000 steps
    against the long-double build of the oracle (the double build holds
    unshifted populations of about 0.3 and rounds each interpolated link
    once per step; that alone reaches 1.1e-12 of the velocity here)."""
    print(f"case curved pipe {storage}", flush=True)
    n = 24
    case = synth.pipe_case(nx=8, ny=n, nz=n, radius=10.0, center=((n - 1) / 2 + 0.3, (n - 1) / 2 - 0.2), g=1e-6)
    links = synth.wall_links(case.mask, case.periodic)
    wq = (links, synth.wall_distances(case, links))
    dom, f = gpu_run(case, storage, 2000, wall_q=wq)
    dom.close()
    _, _, rho_ref, u_ref = oracle_post(case, 2000, wall_q=wq, long_double=True)
    rho, u = moments_from_post(f, case.g)
    assert eps_u(u, u_ref) < tol
    assert np.max(np.abs(rho - rho_ref)) < tol


def test_pipe_second_order_on_the_gpu():
    """The GPU path reproduces the method's convergence: pipe Poiseuille error
    against the start-up series falls about 4x per halving of the spacing
    with exact wall distances (FP64 storage)."""
    import scipy.special
    lam = scipy.special.jn_zeros(0, 60)
    errs = []
    for R in (5, 10, 20):
        print(f"case curved pipe order R={R}", flush=True)
        n = int(2 * R + 4)
        case = synth.pipe_case(nx=4, ny=n, nz=n, radius=R, center=((n - 1) / 2 + 0.3, (n - 1) / 2 - 0.2))
        links = synth.wall_links(case.mask, case.periodic)
        steps = int(20 * R * R)
        dom, f = gpu_run(case, "f64", steps, wall_q=(links, synth.wall_distances(case, links)))
        xyz = dom.coords()
        dom.close()
        _, u = moments_from_post(f, case.g)
        cy, cz = case.meta["center"]
        # gpu_run returns nodes in the oracle's x-fastest order
        zyx = np.argwhere(case.mask == synth.FLUID)
        r = np.sqrt((zyx[:, 1] - cy) ** 2 + (zyx[:, 0] - cz) ** 2)
        nu, g = case.nu, 1e-6
        ua = g * (R * R - r * r) / (4 * nu)
        for lv in lam:
            ua = ua - 2 * g * R * R / nu * scipy.special.j0(lv * r / R) / (lv ** 3 * scipy.special.j1(lv)) \
                * np.exp(-lv * lv * nu * steps / (R * R))
        errs.append(math.sqrt(((u[:, 0] - ua) ** 2).sum() / (ua ** 2).sum()))
        assert len(xyz) == len(r)
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_aneurysm256_prefix_exact_wall_distances(storage, tol):
    """The 256^3 aneurysm with exact wall distances on every wall link,
    Womersley inlet and zero-pressure outlet: the first 300 steps against the
    oracle."""
    print(f"case curved aneurysm256 {storage}", flush=True)
    case = synth.aneurysm_case(256, seed=0)
    links = synth.wall_links(case.mask, case.periodic)
    wq = (links, synth.wall_distances(case, links))
    dom, f = gpu_run(case, storage, 300, wall_q=wq)
    dom.close()
    _, _, _, u_ref = oracle_post(case, 300, wall_q=wq)
    _, u = moments_from_post(f, case.g)
    assert eps_u(u, u_ref) < tol


@pytest.mark.parametrize("cfg", [(0, 256, 0, 0, 0), (1, 256, 0, 0, 0), (1, 128, 0, 64, 1)])
def test_batch_with_curved_walls_equals_solo(cfg):
    """A batch that mixes curved-wall and plain domains steps each of them
    bit-identically to stepping it alone, with per-step launches and with
    the persistent kernel (the blend runs inside the shared step)."""
    from paper_2101_11107_amd import lbm
    cases = [synth.random_tiny_case(s, nx=31, ny=9, nz=8) for s in (1, 3)] + [synth.aneurysm_case(64, 1)]
    wqs = [_random_q(cases[0], 7), None, (synth.wall_links(cases[2].mask, 0),
                                          synth.wall_distances(cases[2], synth.wall_links(cases[2].mask, 0)))]
    steps = 37
    for storage in ("f64", "f32"):
        print(f"case curved batch {storage} cfg {cfg}", flush=True)
        doms = [lbm.Domain(c, storage=storage, wall_q=w) for c, w in zip(cases, wqs)]
        for d in doms:
            d.init()
        b = lbm.Batch(doms)
        b.set_config(cfg)
        b.step(steps)
        b.status()
        got = [d.populations().cpu().numpy() for d in doms]
        b.close()
        for d in doms:
            d.close()
        for c, w, fb in zip(cases, wqs, got):
            d = lbm.Domain(c, storage=storage, wall_q=w)
            d.init()
            d.step(steps)
            fs = d.populations().cpu().numpy()
            d.close()
            assert np.array_equal(fb, fs)
