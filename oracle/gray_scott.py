"""FP64 CPU oracle for the Gray-Scott two-species model on the same transforms.

TEST INFRASTRUCTURE ONLY (see oracle/ch.py).  The paper's two-species reaction-diffusion example
(appendix "Reaction-diffusion systems", eq. gray-scott), with u = c_A, v = c_B, F the feed rate and
k the kill rate exactly as printed there:
    du/dt = D_u lap u - u v^2 + F (1 - u),    dv/dt = D_v lap v + u v^2 - k v.
(The Pearson form often quoted elsewhere writes the kill term as -(F + k') v; it is the same model
with k = F + k'.)
stepped semi-implicitly with the symbol rule of the appendix: diffusion implicit (S = -D K2 per
species), reaction explicit:
    U' = (U + dt T[R_u]) / (1 + dt D_u K2),   V' = (V + dt T[R_v]) / (1 + dt D_v K2),
i.e. one linear solve (I - dt D L) w' = w + dt R(u, v) per species with the Laplacian L that T
diagonalises.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .ch import T, Tinv, k2_grid

__all__ = ["GSParams", "reaction", "gs_step", "gs_run"]


@dataclass(frozen=True)
class GSParams:
    dx: float = 1.0
    dt: float = 1.0
    Du: float = 0.2
    Dv: float = 0.1
    F: float = 0.04
    k: float = 0.10


def reaction(u, v, p: GSParams):
    """(R_u, R_v) = (-u v^2 + F (1 - u), u v^2 - k v)."""
    uv2 = u * v * v
    return -uv2 + p.F * (1.0 - u), uv2 - p.k * v


def gs_step(u, v, p: GSParams, bc, scheme: str):
    """One semi-implicit step of both species."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    K2 = k2_grid(u.shape, p.dx, bc, scheme)
    ru, rv = reaction(u, v, p)
    un = Tinv((T(u, bc) + p.dt * T(ru, bc)) / (1.0 + p.dt * p.Du * K2), bc)
    vn = Tinv((T(v, bc) + p.dt * T(rv, bc)) / (1.0 + p.dt * p.Dv * K2), bc)
    return un, vn


def gs_run(u0, v0, nsteps: int, p: GSParams, bc, scheme: str):
    u, v = np.asarray(u0, np.float64).copy(), np.asarray(v0, np.float64).copy()
    for _ in range(nsteps):
        u, v = gs_step(u, v, p, bc, scheme)
    return u, v
