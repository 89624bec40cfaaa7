"""Pins of the oracle's exponential (ETD1) stepper, each against something other than the
stepper itself: the exponential of the linearised flow (the split for which ETD1 is exact), the
closed-form growth factor, first-order agreement with the semi-implicit step, the scalar phi1
against its series and a direct quadrature, fixed points and mass."""
import numpy as np
import pytest

from oracle import ch
from oracle.ch import CHParams
from paper_2507_21748_amd.inputs import mode_field, quench_field

BCS = ["periodic", "zero_flux"]
SCHEMES = ["spectral", "stencil7"]


def test_phi1_against_series_and_quadrature():
    """phi1(z) = int_0^1 exp(z s) ds: Simpson quadrature on a fine grid, the Taylor series near 0,
    and phi1(0) = 1 exactly."""
    s = np.linspace(0.0, 1.0, 20001)
    for z in [-50.0, -3.0, -0.7, -1e-3, 0.4]:
        w = np.ones_like(s)
        w[1:-1:2], w[2:-1:2] = 4.0, 2.0
        quad = np.sum(w * np.exp(z * s)) * (s[1] - s[0]) / 3.0
        assert abs(float(ch.phi1(z)) / quad - 1.0) < 1e-10
    for z in [-1e-6, 1e-8, -3e-10]:
        assert abs(float(ch.phi1(z)) - (1.0 + z / 2.0 + z * z / 6.0)) < 1e-15
    assert float(ch.phi1(0.0)) == 1.0


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_exact_for_linearised_flow(bc, scheme):
    """With the stabilisation A = M f''(cbar) the split's linear part S equals the linearised
    right-hand side of a small mode on cbar, the remainder N vanishes for it, and ETD1 advances the
    mode by the exact exp(dt lam), lam = -M K2 (f''(cbar) + kappa K2) (to O(delta^2))."""
    cbar, delta, m = 0.8, 1e-7, (0, 1, 1)
    p = CHParams(dt=2.0, A=1.0 * ch.fsecond(cbar))
    shape = (8, 12, 16)
    mode = mode_field(shape, 0.0, 1.0, m, bc).astype(np.float64)
    c = cbar + delta * mode
    n = 5
    for _ in range(n):
        c = ch.ch_step_etd1(c, p, bc, scheme)
    amp = np.sum((c - cbar) * mode) / np.sum(mode * mode)
    K2 = sum(ch.axis_k2(s_, p.dx, bc, scheme)[mi] for s_, mi in zip(shape, m))
    lam = -p.M * K2 * (ch.fsecond(cbar) + p.kappa * K2)
    assert abs(amp / (delta * np.exp(n * p.dt * lam)) - 1.0) < 1e-5


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("cbar", [0.0, 0.3])
def test_linear_growth_factor(bc, scheme, cbar):
    """A mode of amplitude 1e-7 grows by the ETD1 factor 1 + dt phi1(dt S) lam per step, which is
    not the semi-implicit factor."""
    p = CHParams(dt=0.5)
    shape, m, n, delta = (8, 12, 16), (1, 1, 2), 6, 1e-7
    mode = mode_field(shape, 0.0, 1.0, m, bc).astype(np.float64)
    c = cbar + delta * mode
    for _ in range(n):
        c = ch.ch_step_etd1(c, p, bc, scheme)
    amp = np.sum((c - cbar) * mode) / np.sum(mode * mode)
    K2 = sum(ch.axis_k2(s_, p.dx, bc, scheme)[mi] for s_, mi in zip(shape, m))
    g = 1.0 + p.dt * float(ch.phi1(-p.dt * (p.M * p.kappa * K2 ** 2 + p.A * K2))) * \
        (-p.M * K2 * (ch.fsecond(cbar) + p.kappa * K2))
    assert abs(amp / (delta * g ** n) - 1.0) < 1e-5
    assert abs(float(ch.growth_factor_etd1(K2, cbar, p)) / g - 1.0) < 1e-14
    assert abs(float(ch.growth_factor(K2, cbar, p)) / g - 1.0) > 1e-3


@pytest.mark.parametrize("bc", BCS)
def test_first_order_agreement_with_semi_implicit(bc):
    """One ETD1 step and one semi-implicit step from the same state agree to O(dt^2): halving dt
    divides their difference by about 4 (dt small enough that |dt S| < 0.1 on every mode)."""
    c0 = quench_field((8, 8, 12), 0.1, 0.3, seed=5).astype(np.float64)
    diffs = []
    for dt in [1e-4, 5e-5, 2.5e-5]:
        p = CHParams(dt=dt)
        d = ch.ch_step_etd1(c0, p, bc, "spectral") - ch.ch_step(c0, p, bc, "spectral")
        diffs.append(np.linalg.norm(d))
    r = np.log2(np.array(diffs[:-1]) / np.array(diffs[1:]))
    assert np.all(np.abs(r - 2.0) < 0.1)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_mass_and_fixed_points(bc, scheme):
    """The mean is conserved (K2 = 0 leaves the DC bin unchanged) and c = +-1 are fixed points."""
    p = CHParams(dt=1.0)
    c0 = quench_field((8, 10, 12), 0.2, 0.5, seed=6).astype(np.float64)
    c = ch.ch_run_etd1(c0, 10, p, bc, scheme)
    assert abs(c.mean() - c0.mean()) < 1e-13
    for v in (1.0, -1.0):
        one = np.full((6, 8, 10), v)
        assert np.max(np.abs(ch.ch_step_etd1(one, p, bc, scheme) - v)) < 1e-13
