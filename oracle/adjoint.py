"""FP64 CPU oracle for gradients through the semi-implicit CH stepper.

TEST INFRASTRUCTURE ONLY (see oracle/ch.py).  Backpropagation through the solver for inverse
problems and parameter estimation is a capability the paper's Statement of Need claims for the
framework; here it is written out as the discrete adjoint of the k-space step.

One step is c^{n+1} = A c^n - B f'(c^n) with the symmetric operators
    A = T^{-1} diag(G P) T,   B = T^{-1} diag(dt M K2 G) T.
For the loss L = sum_voxels (c^T - c_target)^2:
    lam^T = 2 (c^T - c_target)
    lam^n = A lam^{n+1} - f''(c^n) * (B lam^{n+1}),        dL/dc^0 = lam^0
    dL/dkappa += < lam^{n+1}, T^{-1}[ -dt M K2^2 G C^{n+1} ] >
    dL/dM     += < lam^{n+1}, T^{-1}[ -dt kappa K2^2 G C^{n+1} - dt K2 G F^n ] >
with C^{n+1} = T[c^{n+1}], F^n = T[f'(c^n)].  (The stabilisation A dt K2 does not carry M, so it
contributes nothing to dL/dM.)
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np

from .ch import CHParams, T, Tinv, ch_step, fprime, fsecond, k2_grid

__all__ = ["loss", "forward_trajectory", "adjoint_gradients", "loss_of_params",
           "loss_tangent"]


def loss(cT, target) -> float:
    d = np.asarray(cT, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.sum(d * d))


def forward_trajectory(c0, nsteps: int, p: CHParams, bc: str, scheme: str):
    c = np.asarray(c0, dtype=np.float64).copy()
    traj = [c]
    for _ in range(nsteps):
        c = ch_step(c, p, bc, scheme)
        traj.append(c)
    return traj


def adjoint_gradients(c0, target, nsteps: int, p: CHParams, bc: str, scheme: str):
    """Returns (loss, dL/dc0, dL/dkappa, dL/dM), all FP64, storing every state."""
    traj = forward_trajectory(c0, nsteps, p, bc, scheme)
    K2 = k2_grid(traj[0].shape, p.dx, bc, scheme)
    K4 = K2 * K2
    P = 1.0 + p.A * p.dt * K2
    G = 1.0 / (1.0 + p.dt * p.M * p.kappa * K4 + p.A * p.dt * K2)
    target = np.asarray(target, dtype=np.float64)
    L = loss(traj[-1], target)
    lam = 2.0 * (traj[-1] - target)
    dk = 0.0
    dM = 0.0
    for n in range(nsteps - 1, -1, -1):
        cn, cn1 = traj[n], traj[n + 1]
        Cn1 = T(cn1, bc)
        Fn = T(fprime(cn), bc)
        dk += float(np.sum(lam * Tinv(-p.dt * p.M * K4 * G * Cn1, bc)))
        dM += float(np.sum(lam * Tinv(-p.dt * p.kappa * K4 * G * Cn1 - p.dt * K2 * G * Fn, bc)))
        Lh = T(lam, bc)
        lam = Tinv(G * P * Lh, bc) - fsecond(cn) * Tinv(p.dt * p.M * K2 * G * Lh, bc)
    return L, lam, dk, dM


def loss_of_params(c0, target, nsteps, p: CHParams, bc, scheme) -> float:
    c = np.asarray(c0, dtype=np.float64)
    for _ in range(nsteps):
        c = ch_step(c, p, bc, scheme)
    return loss(c, target)


def loss_tangent(c0, target, nsteps, p: CHParams, bc, scheme, dkappa=0.0, dM=0.0,
                 dc0=None) -> float:
    """Forward-mode (tangent-linear) directional derivative of the loss along
    (dc0, dkappa, dM), carried step by step as value/derivative pairs (dual numbers, exact to
    round-off).  Independent of the reverse sweep in adjoint_gradients:
        C = T c, F = T f'(c), D = 1 + dt M kappa K2^2 + A dt K2, N = P C - dt M K2 F,
        dD = dt K2^2 (dM kappa + M dkappa), dN = P dC - dt dM K2 F - dt M K2 T[f''(c) dc],
        c' = T^{-1}[N / D],  dc' = T^{-1}[dN / D - N dD / D^2]."""
    c = np.asarray(c0, dtype=np.float64).copy()
    dc = np.zeros_like(c) if dc0 is None else np.asarray(dc0, dtype=np.float64).copy()
    K2 = k2_grid(c.shape, p.dx, bc, scheme)
    K4 = K2 * K2
    P = 1.0 + p.A * p.dt * K2
    D = 1.0 + p.dt * p.M * p.kappa * K4 + p.A * p.dt * K2
    dD = p.dt * K4 * (dM * p.kappa + p.M * dkappa)
    for _ in range(nsteps):
        C, dC = T(c, bc), T(dc, bc)
        F, dF = T(fprime(c), bc), T(fsecond(c) * dc, bc)
        N = P * C - p.dt * p.M * K2 * F
        dN = P * dC - p.dt * dM * K2 * F - p.dt * p.M * K2 * dF
        c, dc = Tinv(N / D, bc), Tinv(dN / D - N * dD / (D * D), bc)
    return float(2.0 * np.sum((c - np.asarray(target, dtype=np.float64)) * dc))


def perturbed(p: CHParams, **kw) -> CHParams:
    return replace(p, **kw)
