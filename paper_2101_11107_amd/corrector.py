"""The learned coarse-to-fine corrector: data, training, evaluation, fallback.

Sec. 3.4 runs the aneurysm at twice the grid spacing with acoustic scaling
(time step doubled with it, so lattice velocities are the same on both
grids), scores the coarse field against the fine one with the similarity
index of Eq. (11) and reports the saving in run time.  Here a small U-net
(include/lbmnet.h) maps the period-averaged velocity of the coarse run to the
fine grid; it is trained on pairs of runs of seeded synthetic geometries and
scored on held-out geometries against the FP64 fine run, beside the plain
trilinear upsampling of the coarse field.

Every simulation, tensor operation and optimizer step runs in the library's
HIP kernels; this module sequences them and computes the scores (host FP64
reductions over the gathered node values).
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import lbm
from . import net as nn

# Velocities are divided by this scale before they enter the network (the peak
# centre-line speed of the synthetic inlet is close to it).
U_SCALE = 0.05


@dataclass
class Fields:
    """Period-averaged velocity of one run on its dense grid (device tensors)."""
    u: object          # FP32 [D, H, W, 3], divided by U_SCALE
    mask: object       # uint8 [D, H, W]
    xyz: object        # int32 [n, 3] node coordinates (device)
    u_nodes: object    # FP64 [3, n] period average (device), lattice units
    seconds: float     # wall time of the run (stepping and averaging)
    steps: int


def period_average(case, storage: str, steps: int | None = None, scale: float = 1.0 / U_SCALE) -> Fields:
    """Run `case` from rest for one period (or `steps`), averaging u over
    every step (inside the step kernel), then scatter the average onto the
    dense grid."""
    import torch
    steps = case.period if steps is None else steps
    d = lbm.Domain(case, storage=storage)
    d.init()
    d.average(lbm.LBM_AVG_RESET)
    d.average(lbm.LBM_AVG_TRACK)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d.step(steps)
    u_nodes = d.average(lbm.LBM_AVG_READ)
    d.stream.synchronize()
    seconds = time.perf_counter() - t0
    xyz = torch.from_numpy(d.coords()).to(d.device)
    D, H, W = case.mask.shape
    dense = torch.empty((D, H, W, 3), dtype=torch.float32, device=d.device)
    mask = torch.empty((D, H, W), dtype=torch.uint8, device=d.device)
    nn.lbmnet_scatter(u_nodes, xyz, D, H, W, scale, dense, mask, torch.cuda.current_stream().cuda_stream)
    d.close()
    return Fields(dense, mask, xyz, u_nodes, seconds, steps)


@dataclass
class Pair:
    seed: int
    coarse: Fields
    fine: Fields
    fine_case: object = None


def make_pair(seed: int, fine_n: int = 256, fine_storage: str = "f64", coarse_storage: str = "f32") -> Pair:
    from synth import aneurysm_case
    fine_case = aneurysm_case(fine_n, seed)
    coarse_case = aneurysm_case(fine_n // 2, seed)
    return Pair(seed, period_average(coarse_case, coarse_storage), period_average(fine_case, fine_storage),
                fine_case)


@dataclass
class TrainConfig:
    crop: int = 32            # coarse crop edge (fine crop 2 * crop)
    batch: int = 8
    iters: int = 1500
    lr: float = 2e-3
    lr_final: float = 1e-4
    margin: int = 6           # fine voxels next to crop faces left out of the loss
    seed: int = 0
    log_every: int = 100


@dataclass
class TrainResult:
    params: np.ndarray
    losses: list = field(default_factory=list)
    seconds: float = 0.0
    iters: int = 0


def _crop_origin(rng, fluid_zyx, shape, crop):
    """Origin (z, y, x) of a crop centred on a random fluid voxel, kept inside the grid."""
    c = fluid_zyx[int(rng.integers(0, fluid_zyx.shape[0]))]
    return [int(min(max(int(v) - crop // 2, 0), max(s - crop, 0))) for v, s in zip(c, shape)]


def train(pairs: list, cfg: TrainConfig, params: np.ndarray | None = None, log=print) -> TrainResult:
    """Adam on random crops centred on fluid voxels of the training pairs."""
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(cfg.seed)
    c = cfg.crop
    model = nn.Net(cfg.batch, c, c, c, train=True)
    model.set_params(nn.init_params(cfg.seed) if params is None else params)
    xin = torch.empty((cfg.batch, c, c, c, 4), dtype=torch.float32, device=dev)
    tgt = torch.empty((cfg.batch, 2 * c, 2 * c, 2 * c, 3), dtype=torch.float32, device=dev)
    tmask = torch.empty((cfg.batch, 2 * c, 2 * c, 2 * c), dtype=torch.uint8, device=dev)
    fluid = [np.argwhere(p.coarse.mask.cpu().numpy()) for p in pairs]
    shapes = [tuple(p.coarse.mask.shape) for p in pairs]
    res = TrainResult(params=None)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # every crop of the run drawn up front, in the order one iteration at a
    # time would draw them, and copied to the device once: the loop then
    # makes no synchronizing host-to-device copy and the host does not wait
    # for the GPU between steps
    picks_all = np.empty((cfg.iters, cfg.batch), np.int64)
    org_all = np.empty((cfg.iters, cfg.batch, 3), np.int32)
    for it in range(cfg.iters):
        picks_all[it] = rng.integers(0, len(pairs), cfg.batch)
        org_all[it] = [_crop_origin(rng, fluid[k], shapes[k], c) for k in picks_all[it]]
    origins = torch.from_numpy(org_all).to(dev)
    st = model.stream.cuda_stream
    for it in range(cfg.iters):
        model._in()
        for s, k in enumerate(picks_all[it]):
            p = pairs[k]
            nn.lbmnet_crop(p.coarse.u, p.coarse.mask, p.fine.u, p.fine.mask, origins[it, s: s + 1], c, c, c,
                           cfg.margin, xin[s: s + 1], tgt[s: s + 1], tmask[s: s + 1], st)
        want = (it % cfg.log_every == 0) or it == cfg.iters - 1
        loss = model.loss_grad(xin, tgt, tmask, want_loss=want)
        frac = it / max(1, cfg.iters - 1)
        lr = cfg.lr_final + 0.5 * (cfg.lr - cfg.lr_final) * (1.0 + math.cos(math.pi * frac))
        model.adam_step(lr)
        if want:
            res.losses.append((it, loss))
            if log:
                log(f"iter {it} loss {loss:.4e} lr {lr:.2e}")
    model.stream.synchronize()
    res.seconds = time.perf_counter() - t0
    res.iters = cfg.iters
    res.params = model.get_params()
    model.close()
    return res


# ---- evaluation ---------------------------------------------------------------------------

def similarity_index(u_ref: np.ndarray, u_est: np.ndarray) -> float:
    """Mean over nodes of the similarity index of Eq. (11), read with the
    factor 1/2 that maps it into [0, 1]: SI = (1 + cos) / 2 * (1 - | |a| /
    max |a| - |b| / max |b| |).  Nodes where either speed is zero take cos 0."""
    a = np.linalg.norm(u_ref, axis=0)
    b = np.linalg.norm(u_est, axis=0)
    dot = (u_ref * u_est).sum(axis=0)
    den = a * b
    cos = np.where(den > 0, dot / np.where(den > 0, den, 1.0), 0.0)
    amax = a.max() if a.max() > 0 else 1.0
    bmax = b.max() if b.max() > 0 else 1.0
    return float(np.mean(0.5 * (1.0 + cos) * (1.0 - np.abs(a / amax - b / bmax))))


def rel_l2(u_ref: np.ndarray, u_est: np.ndarray) -> float:
    return float(np.linalg.norm(u_est - u_ref) / np.linalg.norm(u_ref))


def plausibility(u_nodes: np.ndarray, xyz: np.ndarray, shape, case) -> dict:
    """Checks of a predicted fine field that need no fine run: the mean
    |div u| over nodes whose six neighbours are fluid (relative to mean |u|),
    and the imbalance of the volume flux up the inlet leg and down the outlet
    leg through the plane y = 3/4 of the leg height."""
    D, H, W = shape
    grid = np.zeros((D, H, W, 3))
    fl = np.zeros((D, H, W), bool)
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    grid[z, y, x] = u_nodes.T
    fl[z, y, x] = True
    inner = fl.copy()
    for ax in range(3):
        inner &= np.roll(fl, 1, ax) & np.roll(fl, -1, ax)
    div = np.zeros((D, H, W))
    for comp, ax in ((0, 2), (1, 1), (2, 0)):
        g = grid[..., comp]
        div += 0.5 * (np.roll(g, -1, ax) - np.roll(g, 1, ax))
    speed = np.linalg.norm(u_nodes, axis=0).mean()
    div_rel = float(np.abs(div[inner]).mean() / max(speed, 1e-30))
    cx = case.meta["torus_center"][0]
    yp = int(0.75 * case.meta["torus_center"][1])
    sl = grid[:, yp, :, 1]
    msk = fl[:, yp, :]
    xs = np.arange(W)[None, :]
    q_in = float(sl[msk & (xs > cx)].sum())
    q_out = float(sl[msk & (xs < cx)].sum())
    imbalance = float(abs(q_in + q_out) / max(abs(q_in), 1e-30))
    return {"div_rel": div_rel, "flux_imbalance": imbalance}


@dataclass
class EvalResult:
    seed: int
    l2_net: float
    l2_tri: float
    si_net: float
    si_tri: float
    checks: dict
    infer_seconds: float
    coarse_seconds: float
    fine_seconds: float


def predict(params: np.ndarray, pair: Pair, model=None):
    """Network and trilinear fields at the fine fluid nodes: ([3, n], [3, n]) host FP64 in
    lattice units, and the inference time (crop, forward, gather)."""
    import torch
    dev = torch.device("cuda:0")
    Dc, Hc, Wc = pair.coarse.mask.shape
    own = model is None
    if own:
        model = nn.Net(1, Dc, Hc, Wc, train=False)
    model.set_params(params)
    st = model.stream.cuda_stream
    xin = torch.empty((1, Dc, Hc, Wc, 4), dtype=torch.float32, device=dev)
    tgt = torch.empty((1, 2 * Dc, 2 * Hc, 2 * Wc, 3), dtype=torch.float32, device=dev)
    tmask = torch.empty((1, 2 * Dc, 2 * Hc, 2 * Wc), dtype=torch.uint8, device=dev)
    origin = torch.zeros((1, 3), dtype=torch.int32, device=dev)
    out = torch.empty((1, 2 * Dc, 2 * Hc, 2 * Wc, 3), dtype=torch.float32, device=dev)
    tri = torch.empty_like(out)
    n = pair.fine.xyz.shape[0]
    u_net = torch.empty((3, n), dtype=torch.float64, device=dev)
    u_tri = torch.empty((3, n), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    model._in()
    nn.lbmnet_crop(pair.coarse.u, pair.coarse.mask, pair.fine.u, pair.fine.mask, origin, Dc, Hc, Wc, 0, xin, tgt,
                   tmask, st)
    nn.lbmnet_forward(model.handle, xin, out)
    nn.lbmnet_gather(out, pair.fine.xyz, 2 * Dc, 2 * Hc, 2 * Wc, U_SCALE, u_net, st)
    model.stream.synchronize()
    seconds = time.perf_counter() - t0
    nn.lbmnet_trilinear(xin, 1, Dc, Hc, Wc, tri, st)
    nn.lbmnet_gather(tri, pair.fine.xyz, 2 * Dc, 2 * Hc, 2 * Wc, U_SCALE, u_tri, st)
    model.stream.synchronize()
    if own:
        model.close()
    return u_net.cpu().numpy(), u_tri.cpu().numpy(), seconds


def evaluate(params: np.ndarray, pair: Pair, model=None) -> EvalResult:
    u_net, u_tri, secs = predict(params, pair, model)
    ref = pair.fine.u_nodes.cpu().numpy()
    xyz = pair.fine.xyz.cpu().numpy()
    checks = plausibility(u_net, xyz, pair.fine_case.mask.shape, pair.fine_case)
    return EvalResult(pair.seed, rel_l2(ref, u_net), rel_l2(ref, u_tri), similarity_index(ref, u_net),
                      similarity_index(ref, u_tri), checks, secs, pair.coarse.seconds, pair.fine.seconds)


def calibrate(train_evals: list, factor: float = 1.5) -> dict:
    """Fallback thresholds: `factor` times the largest value of each check on
    the training geometries."""
    keys = train_evals[0].checks.keys()
    return {k: factor * max(e.checks[k] for e in train_evals) for k in keys}


def _exceeds(checks: dict, thresholds: dict) -> bool:
    # a non-finite check (a non-finite prediction) fails as well
    return any(not (checks[k] <= thresholds[k]) for k in thresholds)


def falls_back(ev: EvalResult, thresholds: dict) -> bool:
    return _exceeds(ev.checks, thresholds)


def corrected_field(u_net: np.ndarray, pair: Pair, thresholds: dict):
    """The answer for a geometry: the network's fine field [3, n] at the fine
    fluid nodes, unless it is not finite or one of its plausibility checks
    exceeds its threshold; then the fine run itself (the fallback).  Returns
    (field, checks, fell_back)."""
    xyz = pair.fine.xyz.cpu().numpy()
    checks = plausibility(u_net, xyz, pair.fine_case.mask.shape, pair.fine_case)
    fell_back = (not np.isfinite(u_net).all()) or _exceeds(checks, thresholds)
    field = pair.fine.u_nodes.cpu().numpy() if fell_back else u_net
    return field, checks, fell_back


def run_protocol(train_seeds, test_seeds, cfg: TrainConfig, log=print) -> dict:
    """Data generation, training, held-out evaluation and fallback; a summary dict."""
    t0 = time.perf_counter()
    pairs_train = [make_pair(s) for s in train_seeds]
    pairs_test = [make_pair(s) for s in test_seeds]
    t_data = time.perf_counter() - t0
    log(f"data: {len(pairs_train)} + {len(pairs_test)} pairs in {t_data:.1f} s")
    tr = train(pairs_train, cfg, log=log)
    log(f"training: {tr.iters} iterations in {tr.seconds:.1f} s")
    Dc, Hc, Wc = pairs_test[0].coarse.mask.shape
    model = nn.Net(1, Dc, Hc, Wc, train=False)
    ev_train = [evaluate(tr.params, p, model) for p in pairs_train[: min(len(pairs_train), 16)]]
    thr = calibrate(ev_train)
    ev_test = [evaluate(tr.params, p, model) for p in pairs_test]
    model.close()
    # run time of the fine run in the coarse run's storage type, for the speed comparison
    from synth import aneurysm_case
    fine_f32 = [period_average(aneurysm_case(2 * Dc, s), "f32").seconds for s in list(test_seeds)[:2]]
    fb = [falls_back(e, thr) for e in ev_test]
    # with a fallback the fine run is the answer (corrected_field): zero
    # error against itself
    l2_eff = [0.0 if f else e.l2_net for e, f in zip(ev_test, fb)]
    return {
        "train_seeds": list(train_seeds), "test_seeds": list(test_seeds),
        "train_iters": tr.iters, "train_seconds": tr.seconds, "data_seconds": t_data,
        "loss_first": tr.losses[0][1], "loss_last": tr.losses[-1][1],
        "l2_net": [e.l2_net for e in ev_test], "l2_tri": [e.l2_tri for e in ev_test],
        "si_net": [e.si_net for e in ev_test], "si_tri": [e.si_tri for e in ev_test],
        "mean_l2_net": float(np.mean([e.l2_net for e in ev_test])),
        "mean_l2_tri": float(np.mean([e.l2_tri for e in ev_test])),
        "mean_si_net": float(np.mean([e.si_net for e in ev_test])),
        "mean_si_tri": float(np.mean([e.si_tri for e in ev_test])),
        "thresholds": thr, "fallback": fb, "fallback_rate": float(np.mean(fb)),
        "mean_l2_with_fallback": float(np.mean(l2_eff)),
        "infer_seconds": float(np.mean([e.infer_seconds for e in ev_test])),
        "coarse_seconds": float(np.mean([e.coarse_seconds for e in ev_test])),
        "fine_seconds_f64": float(np.mean([e.fine_seconds for e in ev_test])),
        "fine_seconds_f32": float(np.mean(fine_f32)),
        "speedup_vs_fine_f32": float(np.mean(fine_f32) / (np.mean([e.coarse_seconds + e.infer_seconds
                                                                  for e in ev_test]))),
        "train_checks": [e.checks for e in ev_train], "test_checks": [e.checks for e in ev_test],
        "params": tr.params,
    }


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="train and score the coarse-to-fine corrector")
    ap.add_argument("--train", type=int, default=48, help="training seeds 0..train-1")
    ap.add_argument("--test", type=int, default=16, help="held-out seeds after the training seeds")
    ap.add_argument("--iters", type=int, default=6000)
    ap.add_argument("--out", default=None, help="write the summary (JSON) and parameters (.npy) here")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run a plain device copy of this size first (profile counter calibration)")
    a = ap.parse_args(argv)
    if a.copy_probe_mib:
        import torch
        src = torch.empty(a.copy_probe_mib << 20, dtype=torch.uint8, device="cuda:0")
        torch.empty_like(src).copy_(src)
        torch.cuda.synchronize()
    cfg = TrainConfig(iters=a.iters, log_every=max(1, a.iters // 10))
    res = run_protocol(range(a.train), range(a.train, a.train + a.test), cfg,
                       log=lambda m: print(m, flush=True))
    params = res.pop("params")
    print(json.dumps(res))
    if a.out:
        with open(a.out + ".json", "w") as f:
            json.dump(res, f, indent=1)
        np.save(a.out + ".npy", params)


if __name__ == "__main__":
    main()
