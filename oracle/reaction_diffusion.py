"""FP64 CPU oracle for the single-species reaction-diffusion problem on the same transforms.

TEST INFRASTRUCTURE ONLY (see oracle/ch.py).  The paper's reaction-diffusion equation (appendix
"Reaction-diffusion systems", eq. reaction-diffusion) with a constant diffusivity D and a
reaction that depends on the concentration only, here a cubic polynomial
    dc/dt = D lap c + f(c),   f(c) = a0 + a1 c + a2 c^2 + a3 c^3
(a linear source or decay, logistic growth r c (1 - c), a bistable c - c^3, ...).  It is stepped
with the symbol rule of the appendix: the diffusion operator's symbol S_D = -D K2 is implicit, the
reaction explicit; an optional linear stabilisation A (the constant-coefficient splitting of the
same appendix applied to the reaction, S = -(D K2 + A), N = f(c) + A c) gives
    C' = ((1 + A dt) C + dt T[f(c)]) / (1 + A dt + dt D K2),
i.e. one linear solve ((1 + A dt) I - dt D L) c' = (1 + A dt) c + dt f(c) per step with the
Laplacian L that T diagonalises.  With A = 0 it is the appendix's increment form
c' = c + T^{-1}[dt / (1 + dt D K2) T[D L c + f(c)]].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .ch import T, Tinv, k2_grid

__all__ = ["RDParams", "reaction", "rd_step", "rd_run", "rd_growth_factor"]


@dataclass(frozen=True)
class RDParams:
    dx: float = 1.0
    dt: float = 0.5
    D: float = 1.0
    A: float = 0.0
    a0: float = 0.0
    a1: float = 1.0
    a2: float = -1.0   # default reaction: logistic growth c (1 - c)
    a3: float = 0.0


def reaction(c, p: RDParams):
    """f(c) = a0 + a1 c + a2 c^2 + a3 c^3."""
    return p.a0 + p.a1 * c + p.a2 * c * c + p.a3 * c * c * c


def rd_step(c, p: RDParams, bc, scheme: str):
    """One semi-implicit step: C' = ((1 + A dt) C + dt T[f(c)]) / (1 + A dt + dt D K2)."""
    c = np.asarray(c, dtype=np.float64)
    K2 = k2_grid(c.shape, p.dx, bc, scheme)
    P = 1.0 + p.A * p.dt
    return Tinv((P * T(c, bc) + p.dt * T(reaction(c, p), bc)) / (P + p.dt * p.D * K2), bc)


def rd_run(c0, nsteps: int, p: RDParams, bc, scheme: str):
    c = np.asarray(c0, np.float64).copy()
    for _ in range(nsteps):
        c = rd_step(c, p, bc, scheme)
    return c


def rd_growth_factor(K2, p: RDParams):
    """Per-step factor of a mode with eigenvalue K2 under a linear reaction f = a1 c (a0 = a2 =
    a3 = 0): the step is then linear and exact per mode, (1 + A dt + a1 dt) / (1 + A dt + dt D K2).
    """
    P = 1.0 + p.A * p.dt
    return (P + p.a1 * p.dt) / (P + p.dt * p.D * np.asarray(K2, dtype=np.float64))
