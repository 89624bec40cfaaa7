"""Pins of the variable-mobility Cahn-Hilliard oracle:
  * brute force: the right-hand side from per-voxel, per-face loops over the definition;
  * the constant-mobility reduction: with M = const and c = 2 phi - 1 the equation is the
    constant-mobility CH of oracle/ch.py with M_c = 9 M gamma0 / eps, kappa = 2 eps^2 / 9, A = 0,
    so on the 7-point scheme one step of each must agree;
  * exact invariants: mass conservation and uniform fields as fixed points;
  * closed-form decay or growth of a small mode around a uniform phi0;
  * a dense brute-force solve of the increment's linear system."""
import itertools

import numpy as np
import pytest

from oracle import ch, ch_varmob as vm
from paper_2507_21748_amd.inputs import mode_field, quench_field
from tests.test_oracle_ch import _dense_laplacian

BCS = ["periodic", "zero_flux", ("zero_flux", "periodic", "zero_flux")]
SCHEMES = ["spectral", "stencil7"]


def _field(shape, seed):
    return quench_field(shape, 0.5, 0.2, seed=seed).astype(np.float64)


def _rhs_by_loops(phi, p, bcs):
    """rhs from the definition, one voxel and one face at a time."""
    shape = phi.shape

    def nb(idx, ax, step):
        j = list(idx)
        j[ax] += step
        if bcs[ax] == "periodic":
            j[ax] %= shape[ax]
        else:  # mirrored ghost: the edge cell itself
            j[ax] = min(max(j[ax], 0), shape[ax] - 1)
        return tuple(j)

    def g(x):
        return (18.0 / p.eps) * x * (1.0 - x) * (1.0 - 2.0 * x)

    mu = np.zeros(shape)
    for idx in itertools.product(*map(range, shape)):
        lap = 0.0
        for ax in range(3):
            lap += phi[nb(idx, ax, 1)] + phi[nb(idx, ax, -1)] - 2.0 * phi[idx]
        mu[idx] = p.gamma0 * g(phi[idx]) - 2.0 * p.gamma0 * p.eps * lap / p.dx ** 2
    out = np.zeros(shape)
    for idx in itertools.product(*map(range, shape)):
        acc = 0.0
        for ax in range(3):
            for step in (1, -1):
                j = nb(idx, ax, step)
                m_face = 0.5 * p.D0 * (phi[idx] * (1 - phi[idx]) + phi[j] * (1 - phi[j]))
                acc += m_face * (mu[j] - mu[idx])
        out[idx] = acc / p.dx ** 2
    return out


@pytest.mark.parametrize("bc", BCS)
def test_rhs_matches_loops(bc):
    p = vm.VMParams(dx=0.7, D0=1.3, gamma0=0.8, eps=1.5)
    phi = _field((3, 4, 5), 31)
    ref = _rhs_by_loops(phi, p, ch.axis_bcs(bc))
    assert np.max(np.abs(vm.rhs(phi, p, bc) - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("bc", BCS)
def test_constant_mobility_reduces_to_ch(bc):
    p = vm.VMParams(dx=0.9, dt=0.3, gamma0=0.7, eps=1.6, M0=0.4)
    phi = _field((6, 8, 10), 32)
    mc = 9.0 * p.M0 * p.gamma0 / p.eps
    q = ch.CHParams(dx=p.dx, dt=p.dt, M=mc, kappa=2.0 * p.eps ** 2 / 9.0, A=0.0)
    out = vm.vm_step(phi, p, bc, "stencil7", mobility_fn=lambda x: np.full_like(x, p.M0))
    ref = ch.ch_step(2.0 * phi - 1.0, q, bc, "stencil7")
    assert np.max(np.abs((2.0 * out - 1.0) - ref)) < 1e-12


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_mass_conserved_and_uniform_fixed_point(bc, scheme):
    p = vm.VMParams(dt=0.2)
    phi = _field((6, 8, 10), 33)
    out = vm.vm_run(phi, 5, p, bc, scheme)
    assert abs(out.sum() - phi.sum()) < 1e-10
    assert np.max(np.abs(out - phi)) > 1e-3  # it did move
    for v in (0.0, 0.3, 0.5, 1.0):
        u = np.full((4, 6, 8), v)
        assert np.max(np.abs(vm.vm_step(u, p, bc, scheme) - v)) < 1e-15


@pytest.mark.parametrize("bc", ["periodic", "zero_flux"])
@pytest.mark.parametrize("scheme", SCHEMES)
def test_small_mode_in_closed_form(bc, scheme):
    """Around a uniform phi0, grad mu0 = 0, so to first order a mode of 7-point eigenvalue K2h
    obeys d delta/dt = -M(phi0) K2h (gamma0 g'(phi0) + 2 gamma0 eps K2h) delta; one step
    multiplies it by 1 + dt r / (1 + 2 dt gamma0 eps M0 K2^2), K2 of the plan's scheme."""
    p = vm.VMParams(dx=1.1, dt=0.4, D0=1.2, gamma0=0.9, eps=1.7, M0=0.3)
    shape, m, n, delta = (8, 12, 16), (1, 2, 1), 4, 1e-7
    for phi0 in (0.5, 0.2):  # spinodal (growth) and outside it (decay)
        mode = mode_field(shape, 0.0, 1.0, m, bc).astype(np.float64)
        phi = phi0 + delta * mode
        for _ in range(n):
            phi = vm.vm_step(phi, p, bc, scheme)
        K2h = sum(ch.axis_k2(s, p.dx, bc, "stencil7")[mi] for s, mi in zip(shape, m))
        K2 = sum(ch.axis_k2(s, p.dx, bc, scheme)[mi] for s, mi in zip(shape, m))
        gp = (18.0 / p.eps) * ((1 - 2 * phi0) ** 2 - 2 * phi0 * (1 - phi0))
        r = -p.D0 * phi0 * (1 - phi0) * K2h * (p.gamma0 * gp + 2 * p.gamma0 * p.eps * K2h)
        G = 1 + p.dt * r / (1 + 2 * p.dt * p.gamma0 * p.eps * p.M0 * K2 * K2)
        a = np.sum((phi - phi0) * mode) / np.sum(mode * mode)
        assert abs(a / (delta * G ** n) - 1) < 1e-5


@pytest.mark.parametrize("bc", ["periodic", "zero_flux"])
@pytest.mark.parametrize("scheme", SCHEMES)
def test_step_equals_dense_solve(bc, scheme):
    """phi' - phi solves (I + 2 dt gamma0 eps M0 L^2) d = dt rhs with the scheme's dense L."""
    p = vm.VMParams(dx=0.8, dt=0.5, gamma0=1.2, eps=1.4, M0=0.35)
    phi = _field((4, 6, 4), 34)
    L = _dense_laplacian(phi.shape, p.dx, bc, scheme)
    A = np.eye(L.shape[0]) + 2 * p.dt * p.gamma0 * p.eps * p.M0 * (L @ L)
    d = np.linalg.solve(A, p.dt * _rhs_by_loops(phi, p, (bc, bc, bc)).reshape(-1))
    out = vm.vm_step(phi, p, bc, scheme)
    assert np.max(np.abs(out - (phi + d.reshape(phi.shape)))) < 1e-12


def test_dirichlet_rejected():
    with pytest.raises(ValueError):
        vm.vm_step(np.zeros((4, 4, 4)), vm.VMParams(), "dirichlet", "spectral")
