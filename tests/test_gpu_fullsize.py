"""GPU parity at the benchmark geometries (256^3 and 512^3 synthetic aneurysms).

Both sides start from the same seeded smooth density/velocity field (the
``synth`` generator, evaluated at each side's own node coordinates) and run
the same number of steps in the launch configuration the benchmark uses
(``lbm_step`` with graph replays).  The oracle (tier O2, FP64) runs the whole
geometry.  Bars on eps_u = max|u_gpu - u_oracle| / max|u_oracle|: 1e-12 for
FP64 storage, 1e-5 for FP32; for FP16/BF16 storage the bounds follow from the
storage rounding (see the test docstring).
"""

import numpy as np
import pytest

import synth
from synth.fields import smooth_values
from gpu_util import C, W, oracle_order

pytestmark = pytest.mark.gpu

STEPS = 40
# Reduced-precision bounds.  Each step rounds every stored deviation f - w to
# the storage format (relative half-ulp 2^-11 for FP16, 2^-8 for BF16); the
# velocity error after a few tens of steps is a few times the per-step
# rounding of the largest deviations relative to max|u|.  Measured:
# FP16 ~3e-4, BF16 ~2e-3 at 40 steps; the bounds below leave a margin of ~3.
BOUND = {"f64": 1e-12, "f32": 1e-5, "f16s": 1e-3, "bf16s": 8e-3}


def _init_fields(xyz, seed=7):
    v = smooth_values(xyz, seed, 1.0, components=4)
    rho = 1.0 + 0.01 * v[0]
    u = 0.03 * v[1:4]
    return rho, u


_oracle_cache = {}


def _oracle_u(case, key):
    if key not in _oracle_cache:
        from oracle import o1_dense as o1
        from oracle import o2
        sim = o2.O2Sim(case, nthreads=16)
        rho0, u0 = _init_fields(sim.coords)
        sim.f[...] = o1.equilibrium_product(rho0, u0.T)
        sim.run(STEPS)
        _, u = sim.macroscopic()
        _oracle_cache[key] = u
    return _oracle_cache[key]


@pytest.mark.parametrize("size", [256, 512])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "bf16s"])
def test_fullsize_parity_from_smooth_field(size, storage):
    import torch
    from paper_2101_11107_amd import lbm
    print(f"case aneurysm{size} {storage} {STEPS} steps", flush=True)
    case = synth.aneurysm_case(size, seed=0)
    dom = lbm.Domain(case, storage=storage)
    xyz = dom.coords()
    rho0, u0 = _init_fields(xyz)
    rho_t = torch.tensor(rho0, dtype=torch.float64, device="cuda:0")
    u_t = torch.tensor(np.ascontiguousarray(u0), dtype=torch.float64, device="cuda:0")
    dom.init(rho_t, u_t)
    dom.step(STEPS)
    _, u = dom.moments()
    u = u.cpu().numpy().T[oracle_order(xyz, case.mask)]
    mon = dom.monitors()
    dom.close()
    assert np.isfinite(mon).all()
    ref = _oracle_u(case, size)
    eps = float(np.max(np.abs(u - ref)) / np.max(np.abs(ref)))
    print(f"  eps_u = {eps:.3e}", flush=True)
    assert eps < BOUND[storage]
