"""Writes tests/golden/ch256_<variant>.npz: the FP64 oracle's 256^3 off-critical quench (mean 0.2,
amplitude 0.05, seed 2, dt 0.5, M = kappa = 1, A = 2) sampled at fixed voxels after 1, 10, 100
and 1000 steps, for the periodic-spectral and zero-flux-stencil variants.

Only the oracle and the seeded input generator are called.  The sample is 8192 voxels drawn from
numpy's PCG64(seed 12345) without replacement; the GPU test evaluates its field at the same
voxels and forms the sampled relative L2 error.  Also stored: the full-field L2 norm of each
oracle state and, with --sensitivity, the relative L2 distance to an oracle run started one
float32 ulp away (the attainability of a given FP32 tolerance).

usage: python tests/golden/make_ch256_golden.py [--variant periodic|zero_flux] [--sensitivity]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ch  # noqa: E402
from oracle.ch import CHParams  # noqa: E402
from paper_2507_21748_amd.inputs import WORKLOADS  # noqa: E402

CHECKPOINTS = (1, 10, 100, 1000)
NSAMPLE = 8192


def sample_index(n_voxels: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(12345))
    return np.sort(rng.choice(n_voxels, size=NSAMPLE, replace=False))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--variant", choices=["periodic", "zero_flux"], default="periodic")
    ap.add_argument("--sensitivity", action="store_true")
    ap.add_argument("--workers", type=int, default=os.cpu_count())
    args = ap.parse_args()
    ch.WORKERS = args.workers
    w = WORKLOADS["ch256_periodic" if args.variant == "periodic" else "ch256_zeroflux"]
    p = CHParams(dx=w.dx, dt=w.dt, M=w.M, kappa=w.kappa, A=w.A)
    c0 = w.initial()
    idx = sample_index(c0.size)
    c = c0.astype(np.float64)
    c_pert = np.nextafter(c0, np.float32(np.inf)).astype(np.float64) if args.sensitivity else None
    out = {"index": idx, "steps": np.array(CHECKPOINTS)}
    t0 = time.time()
    for n in range(1, max(CHECKPOINTS) + 1):
        c = ch.ch_step(c, p, w.bc, w.scheme)
        if c_pert is not None:
            c_pert = ch.ch_step(c_pert, p, w.bc, w.scheme)
        if n in CHECKPOINTS:
            out[f"values_{n}"] = c.reshape(-1)[idx].copy()
            out[f"norm_{n}"] = np.array(np.linalg.norm(c))
            out[f"mean_{n}"] = np.array(c.mean())
            if c_pert is not None:
                out[f"sens_{n}"] = np.array(np.linalg.norm(c - c_pert) / np.linalg.norm(c))
            print(f"step {n}: {time.time() - t0:.0f} s", flush=True)
    path = os.path.join(HERE, f"ch256_{args.variant}.npz")
    np.savez_compressed(path, **out)
    print("wrote", path)


if __name__ == "__main__":
    main()
