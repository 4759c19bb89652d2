"""The learned corrector's gain test: trained on the GPU on pairs of coarse
and fine runs of seeded geometries, it must beat the trilinear upsampling of
the coarse field on held-out geometries, both scored against the FP64 fine
run (relative L2 of the period-averaged velocity over the fine fluid nodes).

A reduced protocol (12 training geometries, 1500 Adam steps, 3 held-out
geometries) keeps the test near half a minute; the full protocol (48 / 16
geometries) runs from ``python -m paper_2101_11107_amd.corrector``.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_corrector_beats_trilinear_on_held_out_geometries():
    from paper_2101_11107_amd import corrector as C
    print("case corrector gain: train seeds 0..11, held-out 48..50", flush=True)
    train_pairs = [C.make_pair(s) for s in range(12)]
    test_pairs = [C.make_pair(s) for s in (48, 49, 50)]
    for p in train_pairs[:2] + test_pairs:
        # the coarse and fine runs are the sizes the protocol names
        assert p.coarse.mask.shape == (128, 128, 128) and p.fine.mask.shape == (256, 256, 256)
        assert p.fine.steps == 4000 and p.coarse.steps == 2000
    cfg = C.TrainConfig(iters=1500, log_every=500)
    tr = C.train(train_pairs, cfg, log=lambda m: print("  " + m, flush=True))
    assert tr.losses[-1][1] < 0.2 * tr.losses[0][1]
    ratios = []
    for p in test_pairs:
        ev = C.evaluate(tr.params, p)
        ratios.append(ev.l2_net / ev.l2_tri)
        print(f"  seed {p.seed}: rel L2 net {ev.l2_net:.4f} trilinear {ev.l2_tri:.4f}  "
              f"SI net {ev.si_net:.4f} trilinear {ev.si_tri:.4f}", flush=True)
        assert np.isfinite(ev.l2_net) and ev.l2_tri > 0.01
        assert ev.l2_net < 0.85 * ev.l2_tri
    print(f"  error ratio net / trilinear: mean {np.mean(ratios):.3f}", flush=True)


def test_fallback_replaces_implausible_predictions_by_the_fine_run():
    """The fallback of the corrected coarse run: with thresholds calibrated on
    the training geometries (1.5 times the largest value of each check), the
    network's own fields on those geometries pass, while a held-out prediction
    corrupted three ways (noise that breaks mass conservation, reversed flow
    in the outlet leg, a non-finite value) fails its checks, and the answer
    is then the fine run itself, exactly."""
    from paper_2101_11107_amd import corrector as C
    print("case corrector fallback: train seeds 0..3, held-out 48", flush=True)
    train_pairs = [C.make_pair(s) for s in range(4)]
    test_pair = C.make_pair(48)
    tr = C.train(train_pairs, C.TrainConfig(iters=300, log_every=300), log=lambda m: print("  " + m, flush=True))
    evs = [C.evaluate(tr.params, p) for p in train_pairs]
    thr = C.calibrate(evs)
    for p, e in zip(train_pairs, evs):
        u_net, _, _ = C.predict(tr.params, p)
        field, checks, fell_back = C.corrected_field(u_net, p, thr)
        assert not fell_back and field is u_net, (p.seed, checks, thr)
    u_net, _, _ = C.predict(tr.params, test_pair)
    fine = test_pair.fine.u_nodes.cpu().numpy()
    xyz = test_pair.fine.xyz.cpu().numpy()
    rng = np.random.default_rng(0)
    speed = np.linalg.norm(u_net, axis=0).mean()
    noisy = u_net + rng.normal(0.0, speed, u_net.shape)
    reversed_leg = u_net.copy()
    outlet_leg = xyz[:, 0] < test_pair.fine_case.meta["torus_center"][0]
    reversed_leg[:, outlet_leg] *= -1.0
    broken = u_net.copy()
    broken[1, 17] = np.nan
    for name, bad in (("noise", noisy), ("reversed outlet leg", reversed_leg), ("non-finite", broken)):
        field, checks, fell_back = C.corrected_field(bad, test_pair, thr)
        print(f"  {name}: checks {checks} thresholds {thr} fallback {fell_back}", flush=True)
        assert fell_back, name
        assert np.array_equal(field, fine), name
