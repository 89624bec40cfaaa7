"""Pins of the oracle's adjoint gradients (no GPU): central finite differences of the FP64
forward loss, forward-mode (tangent-linear) derivatives carried as dual numbers through the
steps (exact to round-off and independent of the reverse sweep), the dot-product identity
<J v, w> = <v, J^T w> of one linearised step, and a complex-step derivative of one zero-flux step
(the DCT is a real transform, so real and imaginary parts never mix)."""
import numpy as np
import pytest

from oracle import adjoint, ch
from oracle.ch import CHParams
from paper_2507_21748_amd.inputs import quench_field

CASES = [("periodic", "spectral"), ("zero_flux", "stencil7"), ("periodic", "stencil7"),
         ("zero_flux", "spectral")]


def _setup(bc, scheme, shape=(8, 6, 10), nsteps=12):
    p = CHParams(dt=0.5, M=1.0, kappa=1.0, A=2.0)
    c0 = quench_field(shape, 0.0, 0.05, seed=6).astype(np.float64)
    pt = CHParams(dt=0.5, M=0.8, kappa=1.5, A=2.0)
    target = ch.ch_run(c0, nsteps, pt, bc, scheme)
    return p, c0, target, nsteps


@pytest.mark.parametrize("bc,scheme", CASES)
def test_param_gradients_vs_finite_differences(bc, scheme):
    p, c0, tgt, n = _setup(bc, scheme)
    _, _, dk, dM = adjoint.adjoint_gradients(c0, tgt, n, p, bc, scheme)
    for name, val in (("kappa", dk), ("M", dM)):
        th = getattr(p, name)
        h = 1e-5 * max(1.0, abs(th))
        lp = adjoint.loss_of_params(c0, tgt, n, adjoint.perturbed(p, **{name: th + h}), bc, scheme)
        lm = adjoint.loss_of_params(c0, tgt, n, adjoint.perturbed(p, **{name: th - h}), bc, scheme)
        fd = (lp - lm) / (2 * h)
        assert abs(val - fd) <= 1e-6 * abs(fd), (name, val, fd)


@pytest.mark.parametrize("bc,scheme", CASES)
def test_param_gradients_vs_tangent(bc, scheme):
    p, c0, tgt, n = _setup(bc, scheme)
    _, _, dk, dM = adjoint.adjoint_gradients(c0, tgt, n, p, bc, scheme)
    tk = adjoint.loss_tangent(c0, tgt, n, p, bc, scheme, dkappa=1.0)
    tM = adjoint.loss_tangent(c0, tgt, n, p, bc, scheme, dM=1.0)
    assert abs(dk - tk) <= 1e-10 * abs(tk)
    assert abs(dM - tM) <= 1e-10 * abs(tM)


@pytest.mark.parametrize("bc,scheme", CASES[:2])
def test_c0_gradient_vs_tangent_and_fd(bc, scheme):
    p, c0, tgt, n = _setup(bc, scheme)
    _, g, _, _ = adjoint.adjoint_gradients(c0, tgt, n, p, bc, scheme)
    rng = np.random.default_rng(0)
    for _ in range(3):
        v = rng.standard_normal(c0.shape)
        tv = adjoint.loss_tangent(c0, tgt, n, p, bc, scheme, dc0=v)
        assert abs(np.sum(g * v) - tv) <= 1e-10 * abs(tv)
    # a single component by central differences
    idx = (3, 2, 5)
    e = np.zeros_like(c0)
    e[idx] = 1.0
    h = 1e-6
    fd = (adjoint.loss_of_params(c0 + h * e, tgt, n, p, bc, scheme)
          - adjoint.loss_of_params(c0 - h * e, tgt, n, p, bc, scheme)) / (2 * h)
    assert abs(g[idx] - fd) <= 1e-6 * abs(fd) + 1e-12


@pytest.mark.parametrize("bc,scheme", CASES)
def test_one_step_dot_product(bc, scheme):
    """J v = A v - B (f''(c) v) and J^T w = A w - f''(c) (B w) with the step's symmetric
    operators; <J v, w> = <v, J^T w> to round-off, and J v matches a complex step of the step."""
    p = CHParams(dt=0.5)
    shape = (6, 8, 10)
    rng = np.random.default_rng(1)
    c = quench_field(shape, 0.1, 0.4, seed=9).astype(np.float64)
    v, w = rng.standard_normal(shape), rng.standard_normal(shape)
    K2 = ch.k2_grid(shape, p.dx, bc, scheme)
    P = 1 + p.A * p.dt * K2
    G = 1 / (1 + p.dt * p.M * p.kappa * K2 ** 2 + p.A * p.dt * K2)
    Aop = lambda u: ch.Tinv(G * P * ch.T(u, bc), bc)
    Bop = lambda u: ch.Tinv(p.dt * p.M * K2 * G * ch.T(u, bc), bc)
    Jv = Aop(v) - Bop(ch.fsecond(c) * v)
    JTw = Aop(w) - ch.fsecond(c) * Bop(w)
    assert abs(np.sum(Jv * w) - np.sum(v * JTw)) < 1e-12 * np.sqrt(np.sum(Jv ** 2) * np.sum(w ** 2))
    if bc == "zero_flux":
        h = 1e-30
        cs = ch.ch_step(c + 1j * h * v, p, bc, scheme, keep_complex=True)
        assert np.max(np.abs(np.imag(cs) / h - Jv)) < 1e-12 * np.max(np.abs(Jv))
