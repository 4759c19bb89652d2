"""Full-length runs of the aneurysm configurations.

* 256^3 (Womersley inlet with alpha 3 and a 4000-step period, zero-pressure
  outlet; 20,000 steps, five periods): FP64 and FP32 storage against the CPU
  oracle at the last step.
* 512^3 (the same geometry under acoustic scaling: tau 0.6508, period 8000;
  40,000 steps, five periods): FP64 storage against the oracle on a
  2000-step prefix, and every storage form against the FP64 run over the
  whole 40,000 steps (final and last-period-averaged velocity, mass).

The two oracle comparisons take minutes of host time and are marked slow.
"""

import os

import numpy as np
import pytest

import synth
from gpu_util import eps_u, oracle_order

pytestmark = pytest.mark.gpu


def _gpu_u(case, storage, steps):
    from paper_2101_11107_amd import lbm
    dom = lbm.Domain(case, storage=storage)
    print(f"  {storage}: {'in place' if dom.in_place() else 'pull'}", flush=True)
    dom.init()
    dom.step(steps)
    rho, u = dom.moments()
    perm = oracle_order(dom.coords(), case.mask)
    rho, u = rho.cpu().numpy()[perm], u.cpu().numpy()[:, perm].T
    dom.close()
    return rho, u


def _oracle_u(case, steps, chunk=2000):
    from oracle import o2
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)
    sim = o2.O2Sim(case, nthreads=threads)
    while sim.t < steps:
        sim.run(min(chunk, steps - sim.t))
        print(f"  oracle at step {sim.t} of {steps}", flush=True)
    rho, u = sim.macroscopic()
    return np.asarray(rho), np.asarray(u)


@pytest.mark.slow
def test_aneurysm256_20000_steps_against_oracle():
    case = synth.aneurysm_case(256, seed=0)
    steps = 20000
    print(f"case aneurysm256 {steps} steps, f64 and f32 against the oracle", flush=True)
    got = {st: _gpu_u(case, st, steps) for st in ("f64", "f32")}
    rho_ref, u_ref = _oracle_u(case, steps)
    for st, tol in (("f64", 1e-12), ("f32", 1e-5)):
        rho, u = got[st]
        e_u, e_rho = eps_u(u, u_ref), float(np.max(np.abs(rho - rho_ref)))
        print(f"  {st}: eps_u {e_u:.3e}  max |rho - rho_ref| {e_rho:.3e}", flush=True)
        assert e_u < tol and e_rho < tol


@pytest.mark.slow
def test_aneurysm512_f64_prefix_against_oracle():
    """The 512^3 geometry over a 2000-step prefix: FP64 (pull) and FP32 (the
    bench's configuration, streamed in place by the automatic choice)."""
    case = synth.aneurysm_case(512, seed=0)
    steps = 2000
    print(f"case aneurysm512 f64 and f32 {steps}-step prefix against the oracle", flush=True)
    got = {st: _gpu_u(case, st, steps) for st in ("f64", "f32")}
    rho_ref, u_ref = _oracle_u(case, steps, chunk=250)
    for st, tol in (("f64", 1e-12), ("f32", 1e-5)):
        rho, u = got[st]
        e_u, e_rho = eps_u(u, u_ref), float(np.max(np.abs(rho - rho_ref)))
        print(f"  {st}: eps_u {e_u:.3e}  max |rho - rho_ref| {e_rho:.3e}", flush=True)
        assert e_u < tol and e_rho < tol


# Bounds of each storage form against the FP64 run after five periods
# (relative L2 velocity error at the last step and of the last-period mean,
# relative mass drift).  Measured at 40,000 steps: f32 6.4e-7 / 4.3e-7 / 3.0e-9,
# f16s 2.5e-3 / 6.4e-4 / 3.9e-5, bf16s 3.1e-2 / 1.1e-2 / 2.8e-3; the bounds
# leave a factor of about 2.5.  Each stored deviation is rounded once per
# step to 2^-24 (FP32), 2^-11 (FP16) or 2^-8 (BF16) of itself, and the flow
# forgets old rounding over a viscous time, so the error settles instead of
# growing with the step count.
PRECISION_BOUNDS = {"f32": (2e-6, 1.5e-6, 1e-8), "f16s": (6e-3, 2e-3, 1e-4), "bf16s": (8e-2, 3e-2, 7e-3)}


def test_aneurysm512_storage_forms_over_40000_steps():
    from paper_2101_11107_amd import precision
    case = synth.aneurysm_case(512, seed=0)
    print("case aneurysm512 storage forms, 40000 steps against f64", flush=True)
    r = precision.study(case, 40000, log=lambda m: print("  " + m, flush=True))
    assert r["average_steps"] == 8000
    for st, (b_final, b_avg, b_mass) in PRECISION_BOUNDS.items():
        row = r[st]
        assert row["finite"]
        assert row["u_rel_l2_final"] < b_final, st
        assert row["u_rel_l2_period_avg"] < b_avg, st
        assert row["mass_drift"] < b_mass, st
