"""Pins of the single-species reaction-diffusion oracle: a dense brute-force solve of the step's
linear system (Laplacians assembled from closed forms, no transform), the uniform-field map (the
reaction ODE stepped by hand), exact per-mode factors under a linear reaction, the logistic
reaction's fixed points, and the increment form of the appendix for A = 0."""
import numpy as np
import pytest

from oracle import ch, reaction_diffusion as rd
from paper_2507_21748_amd.inputs import mode_field, quench_field
from tests.test_oracle_ch import _dense_laplacian

BCS = ["periodic", "zero_flux"]
SCHEMES = ["spectral", "stencil7"]


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("A", [0.0, 1.5])
def test_step_equals_dense_solve(bc, scheme, A):
    p = rd.RDParams(dx=0.8, dt=0.6, D=0.7, A=A, a0=0.05, a1=0.9, a2=-0.4, a3=-1.1)
    c = quench_field((4, 6, 4), 0.3, 0.4, seed=31).astype(np.float64)
    L = _dense_laplacian(c.shape, p.dx, bc, scheme)
    P = 1.0 + A * p.dt
    I = np.eye(L.shape[0])
    v = c.reshape(-1)
    f = p.a0 + p.a1 * v + p.a2 * v ** 2 + p.a3 * v ** 3
    ref = np.linalg.solve(P * I - p.dt * p.D * L, P * v + p.dt * f).reshape(c.shape)
    got = rd.rd_step(c, p, bc, scheme)
    assert np.max(np.abs(got - ref)) < 1e-12


def test_uniform_field_map():
    """K2 = 0 on a uniform field: c' = c + dt f(c) / (1 + A dt), the reaction ODE's step."""
    for A in (0.0, 2.0):
        p = rd.RDParams(dt=0.7, A=A, a0=0.1, a1=-0.3, a2=0.8, a3=-0.5)
        for c0 in (-0.4, 0.2, 0.9):
            c = np.full((4, 6, 8), c0)
            got = rd.rd_step(c, p, "periodic", "spectral")
            f = 0.1 - 0.3 * c0 + 0.8 * c0 ** 2 - 0.5 * c0 ** 3
            assert np.max(np.abs(got - (c0 + p.dt * f / (1 + A * p.dt)))) < 1e-14


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_linear_reaction_mode_factor_is_exact(bc, scheme):
    """f = a1 c: the step is linear, so a mode of any amplitude changes by exactly
    (1 + A dt + a1 dt) / (1 + A dt + dt D K2) per step."""
    p = rd.RDParams(dt=0.5, D=0.8, A=1.0, a0=0.0, a1=-0.3, a2=0.0, a3=0.0)
    shape, m, n = (8, 12, 16), (1, 2, 3), 7
    mode = mode_field(shape, 0.0, 1.0, m, bc).astype(np.float64)
    c = 0.7 * mode
    for _ in range(n):
        c = rd.rd_step(c, p, bc, scheme)
    K2 = sum(ch.axis_k2(s, p.dx, bc, scheme)[mi] for s, mi in zip(shape, m))
    amp = np.sum(c * mode) / np.sum(mode * mode)
    assert abs(amp / (0.7 * rd.rd_growth_factor(K2, p) ** n) - 1) < 1e-12


@pytest.mark.parametrize("bc", BCS)
def test_logistic_fixed_points_and_small_mode_growth(bc):
    """f = r c (1 - c): c = 0 and c = 1 are fixed points; a small mode on c = 0 grows by
    (1 + r dt) / (1 + dt D K2) and one on c = 1 decays by (1 - r dt) / (1 + dt D K2), to first
    order in the amplitude."""
    r = 0.4
    p = rd.RDParams(dt=0.5, D=0.6, a0=0.0, a1=r, a2=-r, a3=0.0)
    shape, m, n, delta = (8, 12, 16), (1, 0, 2), 5, 1e-7
    for base in (0.0, 1.0):
        u = np.full(shape, base)
        assert np.max(np.abs(rd.rd_step(u, p, bc, "spectral") - base)) < 1e-15
    mode = mode_field(shape, 0.0, 1.0, m, bc).astype(np.float64)
    K2 = sum(ch.axis_k2(s, p.dx, bc, "spectral")[mi] for s, mi in zip(shape, m))
    for base, lin in ((0.0, r), (1.0, -r)):
        c = base + delta * mode
        for _ in range(n):
            c = rd.rd_step(c, p, bc, "spectral")
        amp = np.sum((c - base) * mode) / np.sum(mode * mode)
        g = (1 + lin * p.dt) / (1 + p.dt * p.D * K2)
        assert abs(amp / (delta * g ** n) - 1) < 1e-6


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_increment_form_with_stencil_rhs(bc, scheme):
    """A = 0: the step equals the appendix's increment form with the right-hand side
    D L c + f(c) evaluated in real space (stencil7: the 7-point stencil)."""
    p = rd.RDParams(dt=0.4, D=0.9, a0=0.02, a1=0.5, a2=-0.7, a3=0.3)
    c = quench_field((6, 8, 10), 0.2, 0.3, seed=33).astype(np.float64)
    K2 = ch.k2_grid(c.shape, p.dx, bc, scheme)
    rhs = p.D * ch.laplacian(c, p.dx, bc, scheme) + rd.reaction(c, p)
    inc = c + ch.Tinv(p.dt / (1.0 + p.dt * p.D * K2) * ch.T(rhs, bc), bc)
    assert np.max(np.abs(inc - rd.rd_step(c, p, bc, scheme))) < 1e-12
