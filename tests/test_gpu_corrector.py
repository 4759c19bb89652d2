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
