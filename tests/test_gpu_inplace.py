"""In-place (AA-pattern) streaming against the pull step and the oracle.

The in-place mode keeps the same values in other places (slot reversal on
every other step; lbm_set_streaming), so every result is compared with the
pull step bitwise, and with the FP64 oracle at the bars of the pull step
(FP64 populations of the tiny cases within 1e-13; the config-1 pipe's
velocity within 1e-12 in FP64 and 1e-5 in FP32).  Reads of the
state happen after odd and even numbers of in-place steps, so both layouts
are converted back (streamed: the permutation into the other buffer;
reversed: the slot reversal in place).
"""

import numpy as np
import pytest

import synth
from gpu_util import eps_u, moments_from_post, oracle_order, oracle_post

pytestmark = pytest.mark.gpu

# cumulative step counts at which the state is read: odd and even counts,
# single eager steps and 16-step graph replays
CHECKPOINTS = (1, 2, 3, 19, 36, 53)


def _pair(case, storage, **kw):
    from paper_2101_11107_amd import lbm
    a = lbm.Domain(case, storage=storage, streaming="pull", **kw)
    b = lbm.Domain(case, storage=storage, streaming="inplace", **kw)
    a.init()
    b.init()
    return a, b


def _same_bits(x, y):
    import torch
    return x.shape == y.shape and torch.equal(x.view(torch.int64), y.view(torch.int64))


def _run_and_compare(case, storage, checkpoints=CHECKPOINTS, **kw):
    import torch
    a, b = _pair(case, storage, **kw)
    done = 0
    for c in checkpoints:
        a.step(c - done)
        b.step(c - done)
        done = c
        fa, fb = a.populations(), b.populations()
        torch.cuda.synchronize()
        assert _same_bits(fa, fb), f"{storage}: populations differ after {c} steps"
        assert np.isfinite(fa.cpu().numpy()).all()
    ma, mb = a.monitors(), b.monitors()
    assert np.array_equal(np.asarray(ma), np.asarray(mb)), (ma, mb)
    ra, ua = a.moments()
    rb, ub = b.moments()
    torch.cuda.synchronize()
    assert _same_bits(ra, rb) and _same_bits(ua, ub)
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_inplace_equals_pull_tiny(storage, seed):
    """Random walls, ghost cells (inlet and outlet links), periodic axes,
    random rates and force; rows across row-table entries (nx = 31)."""
    print(f"case tiny{seed} nx=31 {storage} inplace", flush=True)
    case = synth.random_tiny_case(seed, nx=31, ny=9, nz=8)
    _run_and_compare(case, storage)


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_inplace_equals_pull_aneurysm(storage):
    """The 128^3 aneurysm (Womersley inlet, pressure outlet, rates one)."""
    print(f"case aneurysm128 {storage} inplace", flush=True)
    case = synth.aneurysm_case(128, seed=0)
    _run_and_compare(case, storage, checkpoints=(16, 33, 64))


def test_inplace_equals_pull_srt2_and_pipe():
    """The SRT comparator on the periodic config-1 pipe (x wraps through
    explicit offsets)."""
    print("case pipe srt2 f64 inplace", flush=True)
    case = synth.pipe_case(nx=64, ny=24, nz=24, radius=10.0, g=1e-6, tau=0.8)
    case.collision = "srt2"
    _run_and_compare(case, "f64", checkpoints=(5, 32, 49))


@pytest.mark.parametrize("seed", [0, 3])
def test_inplace_matches_oracle_f64(seed):
    """Oracle parity of the in-place run itself: 21 steps (ends in the
    streamed layout) and 20 steps (reversed layout)."""
    from paper_2101_11107_amd import lbm
    for steps in (21, 20):
        print(f"case tiny{seed} f64 inplace {steps} steps vs oracle", flush=True)
        case = synth.random_tiny_case(seed, nx=11, ny=9, nz=8)
        dom = lbm.Domain(case, storage="f64", streaming="inplace")
        dom.init()
        dom.step(steps)
        f = dom.populations().cpu().numpy().T.copy()[oracle_order(dom.coords(), case.mask)]
        dom.close()
        _, ref, _, _ = oracle_post(case, steps)
        assert np.max(np.abs(f - ref)) < 1e-13


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_inplace_pipe_poiseuille_2000_steps(storage, tol):
    """Config 1 in place (x periodic through explicit offsets): velocity and
    density after 2000 steps against the long-double oracle, at the bars of
    the pull step."""
    from paper_2101_11107_amd import lbm
    print(f"case pipe {storage} inplace 2000 steps vs oracle", flush=True)
    case = synth.pipe_case()
    dom = lbm.Domain(case, storage=storage, streaming="inplace")
    dom.init()
    dom.step(2000)
    f = dom.populations().cpu().numpy().T.copy()[oracle_order(dom.coords(), case.mask)]
    dom.close()
    _, _, rho_ref, u_ref = oracle_post(case, 2000, long_double=True)
    rho, u = moments_from_post(f, case.g)
    assert eps_u(u, u_ref) < tol
    assert np.max(np.abs(rho - rho_ref)) < tol


def test_inplace_readers_checkpoint_and_mode_switch():
    """Velocity tracking, accumulation, monitoring points, a checkpoint taken
    in the streamed layout and restored into a fresh domain, and a switch
    back to pull: all equal to the pull run."""
    import torch
    from paper_2101_11107_amd import lbm
    print("case tiny1 f32 inplace readers", flush=True)
    case = synth.random_tiny_case(1, nx=31, ny=9, nz=8)
    a, b = _pair(case, "f32")
    fluid = np.argwhere(case.mask == synth.FLUID)[:3][:, ::-1].copy()   # (x, y, z)
    pa = a.set_probes(fluid, 2, 64)
    pb = b.set_probes(fluid, 2, 64)
    for d in (a, b):
        d.average(lbm.LBM_AVG_RESET)
        d.average(lbm.LBM_AVG_TRACK)
        d.step(17)
    ua, ub = a.average(lbm.LBM_AVG_READ), b.average(lbm.LBM_AVG_READ)
    torch.cuda.synchronize()
    assert _same_bits(ua, ub)
    assert _same_bits(pa, pb)
    for d in (a, b):
        d.average(lbm.LBM_AVG_RESET)
        d.step(3)
        d.average(lbm.LBM_AVG_ACCUMULATE)
        d.step(16)
        d.average(lbm.LBM_AVG_ACCUMULATE)
    ua, ub = a.average(lbm.LBM_AVG_READ), b.average(lbm.LBM_AVG_READ)
    torch.cuda.synchronize()
    assert _same_bits(ua, ub)
    # checkpoint after an odd number of in-place steps since the last reader
    for d in (a, b):
        d.step(5)
    sa, sb = a.get_state(), b.get_state()
    assert sa == sb
    c = lbm.Domain(case, storage="f32", streaming="inplace")
    c.set_state(sb)
    for d in (a, b, c):
        d.step(23)
    b.set_streaming("pull")
    for d in (a, b, c):
        d.step(4)
    fa, fb, fc = a.populations(), b.populations(), c.populations()
    torch.cuda.synchronize()
    assert _same_bits(fa, fb) and _same_bits(fa, fc)
    assert np.array_equal(np.asarray(a.monitors()), np.asarray(c.monitors()))
    for d in (a, b, c):
        d.close()


def test_batch_after_inplace_steps():
    """Domains stepped in place, then batched (the batch takes the pull
    layout), then in place again: equal to the same sequence in pull mode."""
    import torch
    from paper_2101_11107_amd import lbm
    print("case batch after inplace f16s", flush=True)
    cases = synth.batch_cases(count=3)
    runs = []
    for mode in ("pull", "inplace"):
        doms = [lbm.Domain(cs, storage="f16s", streaming=mode) for cs in cases]
        for d in doms:
            d.init()
            d.step(7)
        bt = lbm.Batch(doms)
        bt.step(5)
        bt.close()
        for d in doms:
            d.step(9)
        runs.append([d.populations() for d in doms])
        torch.cuda.synchronize()
        for d in doms:
            d.close()
    for fa, fb in zip(*runs):
        assert _same_bits(fa, fb)


def test_inplace_parameter_changes_mid_run():
    """Relaxation, collision operator, inlet and outlet changed between steps
    (each drops the captured graphs) while the buffer is in either in-place
    layout: equal to the same sequence with pull."""
    import torch
    from paper_2101_11107_amd import lbm
    print("case aneurysm128 f32 inplace parameter changes", flush=True)
    case = synth.aneurysm_case(128, seed=0)
    a, b = _pair(case, "f32")
    seq = [
        (17, lambda d: lbm.lbm_set_params(d.handle, case.tau * 1.05, (1.0, 1.2, 0.9, 1.0), case.g)),
        (16, lambda d: lbm.lbm_set_collision(d.handle, "srt2")),
        (33, lambda d: lbm.lbm_set_outlet_pressure(d.handle, case.rho_out * 1.0005)),
        (5, lambda d: lbm.lbm_set_collision(d.handle, "chm_mrt")),
        (19, None),
    ]
    if case.inlet is not None:
        i = case.inlet
        seq.insert(2, (8, lambda d: lbm.lbm_set_inlet_womersley(d.handle, i.axis, i.center, i.radius, i.G0 * 1.1,
                                                                 i.G1, i.omega)))
    for steps, change in seq:
        for d in (a, b):
            d.step(steps)
            if change is not None:
                change(d)
    fa, fb = a.populations(), b.populations()
    torch.cuda.synchronize()
    assert _same_bits(fa, fb)
    assert np.array_equal(np.asarray(a.monitors()), np.asarray(b.monitors()))
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "f16s"])
@pytest.mark.parametrize("seed", [0, 2])
def test_inplace_curved_equals_pull(storage, seed):
    """Curved walls with random wall distances (both rules of the blend, open
    links and periodic axes on the same tiny masks): the in-place run keeps
    each link's own value aside and equals the pull run bitwise."""
    print(f"case tiny{seed} curved {storage} inplace", flush=True)
    case = synth.random_tiny_case(seed, nx=31, ny=9, nz=8)
    links = synth.wall_links(case.mask, case.periodic)
    q = synth.random_wall_distances(links, seed)
    _run_and_compare(case, storage, wall_q=(links, q))


def test_inplace_curved_equals_pull_aneurysm():
    print("case aneurysm128 curved f32 inplace", flush=True)
    case = synth.aneurysm_case(128, seed=0)
    links = synth.wall_links(case.mask, case.periodic)
    _run_and_compare(case, "f32", checkpoints=(16, 33, 64), wall_q=(links, synth.wall_distances(case, links)))


@pytest.mark.parametrize("seed", [0, 2])
def test_inplace_curved_matches_oracle_f64(seed):
    from paper_2101_11107_amd import lbm
    case = synth.random_tiny_case(seed, nx=11, ny=9, nz=8)
    links = synth.wall_links(case.mask, case.periodic)
    q = synth.random_wall_distances(links, seed)
    for steps in (21, 20):
        print(f"case tiny{seed} curved f64 inplace {steps} steps vs oracle", flush=True)
        dom = lbm.Domain(case, storage="f64", streaming="inplace", wall_q=(links, q))
        dom.init()
        dom.step(steps)
        f = dom.populations().cpu().numpy().T.copy()[oracle_order(dom.coords(), case.mask)]
        dom.close()
        _, ref, _, _ = oracle_post(case, steps, wall_q=(links, q))
        assert np.max(np.abs(f - ref)) < 1e-13


@pytest.mark.parametrize("shape", [(9, 1, 3), (9, 2, 3), (7, 2, 2)])
def test_inplace_periodic_axes_of_length_one_and_two(shape):
    """Periodic axes of length 1 or 2: a node's neighbours across them are
    itself or one node on both sides, so the same place is reached through
    two directions.  Each place still has one reader and writer; in place
    equals pull bitwise and the oracle within 1e-13."""
    from paper_2101_11107_amd import lbm
    nx, ny, nz = shape
    print(f"case periodic box {shape} f64 inplace", flush=True)
    rng = np.random.default_rng(nx * 100 + ny * 10 + nz)
    mask = np.full((nz, ny, nx), synth.FLUID, np.uint8)
    mask[rng.random(mask.shape) < 0.2] = synth.SOLID
    mask[0, 0, 0] = synth.FLUID
    case = synth.Case(name="periodic_box", mask=mask, periodic=7, tau=0.7, rates=(1.1, 0.9, 1.2, 1.0),
                      g=(1e-4, -2e-4, 5e-5))
    _run_and_compare(case, "f64", checkpoints=(1, 2, 3, 19, 36))
    steps = 21
    dom = lbm.Domain(case, storage="f64", streaming="inplace")
    dom.init()
    dom.step(steps)
    f = dom.populations().cpu().numpy().T.copy()[oracle_order(dom.coords(), case.mask)]
    dom.close()
    _, ref, _, _ = oracle_post(case, steps)
    assert np.max(np.abs(f - ref)) < 1e-13
