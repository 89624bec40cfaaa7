"""FP64 CPU oracle for the paper's variable-mobility Cahn-Hilliard step.

TEST INFRASTRUCTURE ONLY (see oracle/ch.py).  The paper's second-order phase transformation
(appendix "Phase transformations of first and second order", eq. cahn-hilliard):
    dphi/dt = div(M grad mu),  mu = gamma0 g(phi) - 2 gamma0 eps lap phi,
    M = D0 phi (1 - phi),      g(phi) = (18 / eps) phi (1 - phi) (1 - 2 phi),
stepped with the appendix "Semi-implicit timestepping" in its increment form
    phi' = phi + T^{-1}{ dt / (1 - dt S) T{ rhs(phi) } },  S = -2 gamma0 eps M0 K2^2,
where rhs = div(M grad mu) is the finite-difference right-hand side evaluated in real space and
M0 the constant reference mobility of the splitting M = M0 + (M - M0).

Finite differences (cell-centred grid, spacing dx):
  * lap phi: the 7-point stencil; a periodic axis wraps, a zero-flux axis mirrors the edge cell
    into its ghost (phi_{-1} = phi_0, phi_n = phi_{n-1});
  * div(M grad mu): conservative face fluxes, (1/dx^2) sum over the six faces of
    M_f (mu_nb - mu), with M_f the mean of the two cells' mobilities; mu takes the same ghosts,
    so a zero-flux boundary face carries no flux.
K2 is the eigenvalue of -L for the plan's scheme (spectral or 7-point) and boundaries.

Readings (the paper prints the Cahn-Hilliard prefactor as dt / (1 + 2 dt eps M0 k^4)):
  * the implicit fourth-order symbol keeps gamma0, S = -2 gamma0 eps M0 K2^2 (the linear part of
    div(M0 grad mu)); it equals the printed form at gamma0 = 1;
  * the face mobility is the arithmetic mean of the two adjacent cells' D0 phi (1 - phi);
  * the forcing f of the equation is zero here, and Dirichlet boundaries are not covered (only
    periodic and zero-flux axes, as the stencil's ghosts above).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .ch import T, Tinv, axis_bcs, k2_grid, laplacian

__all__ = ["VMParams", "mobility", "g", "chemical_potential", "div_mobility_grad", "rhs",
           "vm_step", "vm_run"]


@dataclass(frozen=True)
class VMParams:
    dx: float = 1.0
    dt: float = 0.05
    D0: float = 1.0
    gamma0: float = 1.0
    eps: float = 2.0
    M0: float = 0.25


def _check_bc(bc):
    if any(b not in ("periodic", "zero_flux") for b in axis_bcs(bc)):
        raise ValueError("variable-mobility step: periodic or zero-flux axes only")


def mobility(phi, p: VMParams):
    """M = D0 phi (1 - phi)."""
    return p.D0 * phi * (1.0 - phi)


def g(phi, p: VMParams):
    """Homogeneous part of the chemical potential, (18 / eps) phi (1 - phi) (1 - 2 phi)."""
    return (18.0 / p.eps) * phi * (1.0 - phi) * (1.0 - 2.0 * phi)


def chemical_potential(phi, p: VMParams, bc):
    """mu = gamma0 g(phi) - 2 gamma0 eps L phi with the 7-point L."""
    return p.gamma0 * g(phi, p) - 2.0 * p.gamma0 * p.eps * laplacian(phi, p.dx, bc, "stencil7")


def _neighbours(u, ax: int, bca: str):
    """(u at +1, u at -1) along axis ax: periodic wrap or mirrored edge ghosts."""
    if bca == "periodic":
        return np.roll(u, -1, axis=ax), np.roll(u, 1, axis=ax)
    pad = [(0, 0)] * 3
    pad[ax] = (1, 1)
    ue = np.pad(u, pad, mode="edge")
    up = [slice(None)] * 3
    dn = [slice(None)] * 3
    up[ax] = slice(2, None)
    dn[ax] = slice(0, -2)
    return ue[tuple(up)], ue[tuple(dn)]


def div_mobility_grad(mu, mob, dx: float, bc):
    """div(M grad mu) as the sum of the six face fluxes M_f (mu_nb - mu) / dx^2."""
    out = np.zeros_like(mu)
    for ax, bca in enumerate(axis_bcs(bc)):
        mu_up, mu_dn = _neighbours(mu, ax, bca)
        m_up, m_dn = _neighbours(mob, ax, bca)
        out = out + 0.5 * (mob + m_up) * (mu_up - mu) + 0.5 * (mob + m_dn) * (mu_dn - mu)
    return out / (dx * dx)


def rhs(phi, p: VMParams, bc, mobility_fn=None):
    """The real-space right-hand side div(M grad mu).  mobility_fn replaces D0 phi (1 - phi)
    (the constant-mobility reduction is one of the oracle's pins)."""
    _check_bc(bc)
    mu = chemical_potential(phi, p, bc)
    mob = mobility(phi, p) if mobility_fn is None else mobility_fn(phi)
    return div_mobility_grad(mu, mob, p.dx, bc)


def vm_step(phi, p: VMParams, bc, scheme: str, mobility_fn=None):
    """One step of the increment form: phi + T^{-1}[dt / (1 + 2 dt gamma0 eps M0 K2^2) T[rhs]]."""
    K2 = k2_grid(phi.shape, p.dx, bc, scheme)
    mult = p.dt / (1.0 + 2.0 * p.dt * p.gamma0 * p.eps * p.M0 * K2 * K2)
    return phi + Tinv(mult * T(rhs(phi, p, bc, mobility_fn), bc), bc)


def vm_run(phi0, nsteps: int, p: VMParams, bc, scheme: str):
    phi = np.asarray(phi0, dtype=np.float64)
    for _ in range(nsteps):
        phi = vm_step(phi, p, bc, scheme)
    return phi
