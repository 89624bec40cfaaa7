"""Writes tests/golden/inverse128.npz: the FP64 oracle's gradients for the 128^3 inverse problem.

Workload: periodic spectral grid 128^3, c0 = 0.05 U(-1, 1) from seed 5 (mean 0), dt 0.5, A 2,
200 steps.  The target is the oracle's own c^T from the same c0 with kappa 1.5, M 0.8; the loss
L = sum (c^T - target)^2 is evaluated at kappa 1, M 1.  Stored: L, dL/dkappa, dL/dM, the norm
of the target, and dL/dc0 at 8192 voxels (PCG64 seed 12345, without replacement) plus its full
L2 norm.  (The GPU test builds its target with its own solver; the FP32 target differs from this
one by about 1e-6 relative, which moves the gradients far less than the 1e-4 tolerance.)  Only the oracle and the seeded
input generator are called.

usage: python tests/golden/make_inverse128_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import adjoint, ch  # noqa: E402
from oracle.ch import CHParams  # noqa: E402
from paper_2507_21748_amd.inputs import WORKLOADS  # noqa: E402


def main():
    ch.WORKERS = os.cpu_count()
    w = WORKLOADS["inverse128"]
    c0 = w.initial().astype(np.float64)
    pt = CHParams(dt=w.dt, M=w.extra["target_M"], kappa=w.extra["target_kappa"], A=w.A)
    target = ch.ch_run(c0, w.steps, pt, w.bc, w.scheme).astype(np.float32)
    p = CHParams(dt=w.dt, M=w.M, kappa=w.kappa, A=w.A)
    L, g, dk, dM = adjoint.adjoint_gradients(c0, target.astype(np.float64), w.steps, p, w.bc,
                                             w.scheme)
    idx = np.sort(np.random.Generator(np.random.PCG64(12345)).choice(c0.size, 8192, replace=False))
    path = os.path.join(HERE, "inverse128.npz")
    np.savez_compressed(path, loss=L, dkappa=dk, dM=dM, target_norm=np.linalg.norm(target),
                        index=idx,
                        grad_c0_sample=g.reshape(-1)[idx], grad_c0_norm=np.linalg.norm(g))
    print("wrote", path, L, dk, dM)


if __name__ == "__main__":
    main()
