"""Reduced-precision storage over a long run: every storage form of one
geometry stepped the same number of steps on the GPU, compared with the FP64
storage run of the same geometry.

For each form: the relative L2 error of the velocity at the last step and of
the velocity averaged over the last inlet period (the time average of the
paper's resolution study, Sec. 3.4), the largest relative velocity error
over the nodes, and the relative drift of the total mass, each against the
FP64 run.  Only the library runs here; nothing is compared with the CPU
oracle.
"""

from __future__ import annotations

import numpy as np

from . import lbm


def _run(case, storage, steps, period, device):
    dom = lbm.Domain(case, storage=storage, device=device)
    dom.init()
    if steps > period:
        dom.step(steps - period)
    dom.average(lbm.LBM_AVG_RESET)
    dom.average(lbm.LBM_AVG_TRACK)
    dom.step(min(steps, period))
    u_avg = dom.average(lbm.LBM_AVG_READ).cpu().numpy()
    _, u = dom.moments()
    u = u.cpu().numpy()
    mon = dom.monitors()
    n = dom.n
    dom.close()
    return u, u_avg, mon, n


def _rel_l2(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def study(case, steps, period=None, storages=("f32", "f16s", "bf16s"), device="cuda:0", log=None):
    """Run FP64 and each storage form for `steps` steps (averaging over the
    last `period` steps, the case's inlet period by default); returns
    {"fp64": {...}, form: {...}}."""
    period = int(period or case.period or steps)
    u64, a64, m64, n = _run(case, "f64", steps, period, device)
    out = {"steps": int(steps), "average_steps": int(min(steps, period)), "fluid_nodes": int(n),
           "f64": {"mass": float(m64[0]), "u_max": float(np.abs(u64).max())}}
    for st in storages:
        u, a, m, _ = _run(case, st, steps, period, device)
        row = {"u_rel_l2_final": _rel_l2(u, u64), "u_rel_l2_period_avg": _rel_l2(a, a64),
               "u_max_rel_err_final": float(np.abs(u - u64).max() / np.abs(u64).max()),
               "mass_drift": float(abs(m[0] - m64[0]) / m64[0]), "finite": bool(np.isfinite(u).all())}
        out[st] = row
        if log:
            log(f"{case.name} {st} {steps} steps: {row}")
    return out
