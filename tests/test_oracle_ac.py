"""Pins of the oracle's Allen-Cahn steps (semi-implicit and ETD1): a dense brute-force solve of
the semi-implicit linear system with Laplacians assembled from closed-form matrices, the
closed-form growth of a small mode, the uniform-field map (the ODE dc/dt = -M f'(c) stepped by
hand), energy decay, relaxation to the wells, and the exact exponential of the linearised split
for ETD1."""
import numpy as np
import pytest

from oracle import ch
from oracle.ch import CHParams
from paper_2507_21748_amd.inputs import mode_field, quench_field
from tests.test_oracle_ch import _dense_laplacian

BCS = ["periodic", "zero_flux"]
SCHEMES = ["spectral", "stencil7"]


def _dense_ac_step(c, p, bc, scheme):
    L = _dense_laplacian(c.shape, p.dx, bc, scheme)
    I = np.eye(L.shape[0])
    v = c.reshape(-1)
    lhs = (1.0 + p.A * p.dt) * I - p.dt * p.M * p.kappa * L
    rhs = (1.0 + p.A * p.dt) * v - p.dt * p.M * (v ** 3 - v)
    return np.linalg.solve(lhs, rhs).reshape(c.shape)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_step_equals_dense_solve(bc, scheme):
    p = CHParams(dx=0.7, dt=0.3, M=0.8, kappa=1.3, A=2.0)
    c = quench_field((4, 6, 4), 0.1, 0.6, seed=41).astype(np.float64)
    ref = _dense_ac_step(c, p, bc, scheme)
    got = ch.ac_step(c, p, bc, scheme)
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("etd1", [False, True])
def test_uniform_field_map(etd1):
    """A uniform field has K2 = 0 only: semi-implicit c' = c - dt M f'(c) / (1 + A dt); ETD1
    c' = c + dt phi1(-A dt) (-M f'(c)).  Both drive 0.3 and -0.2 to the wells +-1."""
    p = CHParams(dt=0.4, M=1.0, A=2.0)
    for c0 in (0.3, -0.2, 1.0, 0.0):
        c = np.full((4, 4, 6), c0)
        got = ch.ac_step_etd1(c, p, "periodic", "spectral") if etd1 else \
            ch.ac_step(c, p, "periodic", "spectral")
        fp = c0 ** 3 - c0
        want = c0 + p.dt * float(ch.phi1(-p.A * p.dt)) * (-p.M * fp) if etd1 else \
            c0 - p.dt * p.M * fp / (1.0 + p.A * p.dt)
        assert np.max(np.abs(got - want)) < 1e-14
    for c0, well in ((0.3, 1.0), (-0.2, -1.0)):
        c = ch.ac_run(np.full((4, 4, 6), c0), 200, p, "periodic", "spectral", etd1=etd1)
        assert np.max(np.abs(c - well)) < 1e-10


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("etd1", [False, True])
def test_linear_growth_factor(bc, scheme, etd1):
    """A mode of amplitude 1e-7 on the well c = 1 (f' = 0, f'' = 2) decays by g per step."""
    p = CHParams(dt=0.5, M=0.9, kappa=1.2, A=1.5)
    shape, m, n, delta, cbar = (8, 12, 16), (1, 1, 2), 6, 1e-7, 1.0
    mode = mode_field(shape, 0.0, 1.0, m, bc).astype(np.float64)
    c = cbar + delta * mode
    for _ in range(n):
        c = ch.ac_step_etd1(c, p, bc, scheme) if etd1 else ch.ac_step(c, p, bc, scheme)
    amp = np.sum((c - cbar) * mode) / np.sum(mode * mode)
    K2 = sum(ch.axis_k2(s_, p.dx, bc, scheme)[mi] for s_, mi in zip(shape, m))
    g = float(ch.ac_growth_factor(K2, cbar, p, etd1=etd1))
    assert abs(amp / (delta * g ** n) - 1.0) < 1e-5


def test_etd1_exact_for_linearised_flow():
    """A = M f''(cbar) on the well cbar = 1: ETD1 advances a small mode by exp(dt lam),
    lam = -M (f''(1) + kappa K2)."""
    p = CHParams(dt=0.7, M=0.9, kappa=1.2, A=0.9 * ch.fsecond(1.0))
    shape, m, n, delta, bc, scheme = (8, 12, 16), (0, 1, 1), 4, 1e-7, "periodic", "spectral"
    mode = mode_field(shape, 0.0, 1.0, m, bc).astype(np.float64)
    c = 1.0 + delta * mode
    for _ in range(n):
        c = ch.ac_step_etd1(c, p, bc, scheme)
    amp = np.sum((c - 1.0) * mode) / np.sum(mode * mode)
    K2 = sum(ch.axis_k2(s_, p.dx, bc, scheme)[mi] for s_, mi in zip(shape, m))
    lam = -p.M * (ch.fsecond(1.0) + p.kappa * K2)
    assert abs(amp / (delta * np.exp(n * p.dt * lam)) - 1.0) < 1e-6


@pytest.mark.parametrize("bc,scheme", [("periodic", "spectral"), ("zero_flux", "stencil7")])
@pytest.mark.parametrize("etd1", [False, True])
def test_energy_decays(bc, scheme, etd1):
    """Allen-Cahn is the L2 gradient flow of the same free energy: with A = 2 the energy of a
    quench decreases at every step."""
    p = CHParams(dt=0.5, M=1.0, kappa=1.0, A=2.0)
    c = quench_field((12, 12, 16), 0.1, 0.5, seed=42).astype(np.float64)
    e = [ch.energy(c, p, bc, scheme)]
    for _ in range(30):
        c = ch.ac_step_etd1(c, p, bc, scheme) if etd1 else ch.ac_step(c, p, bc, scheme)
        e.append(ch.energy(c, p, bc, scheme))
    assert np.all(np.diff(e) <= 1e-12 * abs(e[0]))
