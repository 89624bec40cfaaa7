"""Learned coarse stepper against plain stepping at equal error.

Trains the network on windows of seeded 256^3 solver trajectories, then rolls a seeded 512^3
quench forward to T = 500 (100 applications of one network step = 10 solver steps of dt 0.5),
judging every prediction with the solver and falling back to it, under both verification modes
of the rollout controller ("window": random one-window spot checks, fast but unverified between
checks; "span": every accepted state verified against the solver's span, sound but at least the
solver's cost).  Reference: the library's FP32 solver at dt 0.5 (itself checked against the
FP64 oracle at 256^3).  Plain candidates: the same solver with dt in {0.5, 1, 2.5, 5}.  The
network wins if its wall time is below that of the fastest plain candidate whose relative L2
error to the reference is <= 1e-2 and its own error is <= 1e-2.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import evx
from .inputs import quench_field
from .surrogate import Net, RolloutConfig, make_pairs, rollout, sample_windows


def _rel(plan, a, b):
    d = plan.distance(a, b).cpu().numpy()
    return float(np.sqrt(d[0] / d[1]))


def train_network(iters: int = 600, batch: int = 4, edge: int = 72, halo: int = 4,
                  lr: float = 1e-3, train_shape=(256, 256, 256), seed: int = 0):
    t0 = time.perf_counter()
    prm = evx.CHParams(dt=0.5)
    pairs = make_pairs(train_shape, [0.0, 0.2], [100, 101], 500, 10, 10, prm)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    rng = np.random.default_rng(seed)
    net = Net(seed=seed)
    losses = []
    t1 = time.perf_counter()
    for it in range(iters):
        x, y = sample_windows(pairs, batch, edge, rng)
        rate = lr * 0.5 * (1 + np.cos(np.pi * it / iters))
        losses.append(float(net.train_step(x, y, halo, rate).item()))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    del pairs
    net.release_workspaces()
    torch.cuda.empty_cache()
    return net, {"data_s": t_data, "train_s": t_train, "iters": iters, "batch": batch,
                 "window": edge, "halo": halo, "loss_first": losses[0],
                 "loss_last10": float(np.mean(losses[-10:]))}


def surrogate_vs_plain(net: Net, shape=(512, 512, 512), napps: int = 100, seed: int = 7):
    prm = evx.CHParams(dt=0.5)
    T = napps * 10 * prm.dt
    plan = evx.Plan(shape, "periodic", "spectral", ops=evx.OP_STEP | evx.OP_DIAG)
    c0 = torch.from_numpy(quench_field(shape, 0.0, 0.05, seed)).cuda()
    out = {"grid": list(shape), "T": T, "applications": napps}
    # reference and plain candidates
    ref = None
    plain = {}
    for dt in (0.5, 1.0, 2.5, 5.0):
        c = c0.clone()
        n = int(round(T / dt))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.step(c, n, evx.CHParams(dt=dt))
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        if ref is None:
            ref = c
        plain[str(dt)] = {"steps": n, "seconds": secs, "rel_l2": _rel(plan, c, ref)}
    out["plain"] = plain
    # network rollouts with the solver as judge and fallback
    net.infer(c0)  # warm-up (workspace allocation, code load)
    ok = [v["seconds"] for v in plain.values() if v["rel_l2"] <= 1e-2]
    out["fastest_plain_within_1e-2_s"] = min(ok) if ok else None
    out["surrogate"] = {}
    for mode in ("window", "span"):
        c, st = rollout(net, c0, napps, prm, RolloutConfig(verify=mode), plan=plan)
        err = _rel(plan, c, ref)
        errs = np.asarray(st.spot_errors, dtype=np.float64)
        out["surrogate"][mode] = {
            "seconds": st.seconds, "rel_l2": err, "accepted": st.accepted,
            "fallback_mass": st.fallback_mass, "fallback_energy": st.fallback_energy,
            "fallback_spot": st.fallback_spot, "spot_checks": st.spot_checks,
            "solver_windows": st.solver_windows,
            "spot_error_min_median_max": ([float(errs.min()), float(np.median(errs)),
                                           float(errs.max())] if errs.size else None),
            "wins": bool(ok and err <= 1e-2 and st.seconds < min(ok))}
    # pure network cost per application (no judging)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tmp = torch.empty_like(c0)
    for _ in range(5):
        net.infer(c0, tmp)
    torch.cuda.synchronize()
    out["network_ms_per_application"] = 1e3 * (time.perf_counter() - t0) / 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tmp.copy_(c0)
    plan.step(tmp, 50, prm)
    torch.cuda.synchronize()
    out["solver_ms_per_10_steps"] = 1e3 * (time.perf_counter() - t0) / 5
    out["surrogate_wins"] = any(v["wins"] for v in out["surrogate"].values())
    return out
