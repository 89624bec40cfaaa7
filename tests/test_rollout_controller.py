"""The coarse-stepper rollout controller's decisions, driven on the CPU by a fake solver built on
the FP64 oracle and by mock networks (no GPU): an exact network is always accepted, a
mass-violating one falls back on mass, an energy-raising one on energy, and a slightly wrong one
is caught by the spot check; every fallback replaces the prediction by the solver's steps.  An
adversarial network, wrong only on the windows a fixed schedule would leave unchecked and
passing the mass and energy checks there, cannot move a span-verified rollout away from the
solver, and is caught by the window-verified one."""
import numpy as np
import torch

from oracle import ch
from paper_2507_21748_amd import evx
from paper_2507_21748_amd.inputs import quench_field
from paper_2507_21748_amd.surrogate import RolloutConfig, rollout


class FakePlan:
    """Solver, diagnostics and distance with the plan's interface, computed by the oracle."""

    def __init__(self, shape):
        self.shape = shape

    def step(self, c, nsteps, prm):
        p = ch.CHParams(dt=prm.dt, M=prm.M, kappa=prm.kappa, A=prm.A)
        out = ch.ch_run(c.numpy().astype(np.float64), nsteps, p, "periodic", "spectral")
        c.copy_(torch.from_numpy(out.astype(np.float32)))
        return c

    def diagnostics(self, c, prm, out=None):
        p = ch.CHParams(dt=prm.dt, M=prm.M, kappa=prm.kappa, A=prm.A)
        c64 = c.numpy().astype(np.float64)
        return torch.tensor([ch.mass(c64), ch.energy(c64, p, "periodic", "spectral")],
                            dtype=torch.float64)

    def distance(self, a, b, out=None):
        a64, b64 = a.numpy().astype(np.float64), b.numpy().astype(np.float64)
        return torch.tensor([np.sum((a64 - b64) ** 2), np.sum(b64 ** 2)], dtype=torch.float64)


class MockNet:
    def __init__(self, plan, kind):
        self.plan, self.kind = plan, kind

    def infer(self, c, out, conserve_mass=False):
        exact = c.clone()
        self.plan.step(exact, 10, evx.CHParams(dt=0.5))
        if self.kind == "exact":
            out.copy_(exact)
        elif self.kind == "mass":
            out.copy_(exact + 1e-3)
        elif self.kind == "energy":
            noise = torch.from_numpy(quench_field(c.shape, 0.0, 1.0, 99)).double()
            out.copy_((c.double() + 0.3 * (noise - noise.mean())).float())   # same mass
        elif self.kind == "slightly_wrong":
            out.copy_(exact * 1.01)
        elif self.kind == "wrong_unchecked":
            # exact on every 10th call (where a fixed schedule checks), otherwise the exact field
            # shifted by one voxel: the same mass and free energy, far from the solver
            self.calls = getattr(self, "calls", 0) + 1
            if (self.calls - 1) % 10 == 0:
                out.copy_(exact)
            else:
                out.copy_(torch.roll(exact, 1, dims=2))
        return out


def _run(kind, napps=6, verify="window", check_every=2):
    shape = (12, 12, 12)
    plan = FakePlan(shape)
    c0 = torch.from_numpy(quench_field(shape, 0.0, 0.05, seed=1))
    cfg = RolloutConfig(check_every=check_every, conserve_mass=False, verify=verify)
    c, st = rollout(MockNet(plan, kind), c0, napps, evx.CHParams(dt=0.5), cfg, plan=plan)
    ref = c0.clone()
    plan.step(ref, 10 * napps, evx.CHParams(dt=0.5))
    return c, ref, st


def test_exact_network_always_accepted():
    for verify in ("window", "span"):
        c, ref, st = _run("exact", verify=verify)
        assert st.accepted == st.applications == 6
        assert st.spot_checks >= 2          # the first and the last application at least
        assert max(st.spot_errors) < 1e-6
        assert torch.allclose(c, ref, atol=1e-5)


def test_mass_violation_falls_back():
    c, ref, st = _run("mass")
    assert st.fallback_mass == 6 and st.accepted == 0
    assert torch.allclose(c, ref, atol=1e-5)


def test_energy_increase_falls_back():
    c, ref, st = _run("energy")
    assert st.fallback_energy == 6 and st.accepted == 0
    assert torch.allclose(c, ref, atol=1e-5)


def test_spot_check_catches_wrong_prediction():
    c, ref, st = _run("slightly_wrong")
    assert st.spot_checks >= 1 and st.fallback_spot >= 1
    assert st.fallback_spot + st.fallback_energy + st.fallback_mass + st.accepted == 6
    # a failing network is checked on every application until one passes: none is accepted
    assert st.accepted == 0
    assert torch.allclose(c, ref, atol=1e-5)


def _rel(a, b):
    a, b = a.double(), b.double()
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def test_span_verification_bounds_an_adversarial_network():
    """Wrong only where a fixed one-in-ten schedule would not look, with mass and energy intact:
    every span check fails and the solver's span replaces the network's, so the rollout ends on
    the solver's trajectory (error within spot_tol, here zero up to FP32)."""
    c, ref, st = _run("wrong_unchecked", napps=23, verify="span", check_every=10)
    assert st.fallback_mass == 0 and st.fallback_energy == 0
    assert st.fallback_spot == st.spot_checks == 3      # spans of 10, 10 and the last 3
    assert _rel(c, ref) <= RolloutConfig().spot_tol
    assert _rel(c, ref) < 1e-6


def test_window_verification_catches_an_adversarial_network():
    """The window mode checks random windows: it finds the wrong predictions, and each failure
    makes it check every following application until one passes."""
    c, ref, st = _run("wrong_unchecked", napps=30, verify="window", check_every=10)
    assert st.fallback_mass == 0 and st.fallback_energy == 0
    assert st.fallback_spot >= 2
    # after a failure the next application is checked too (strict mode): checks come in runs
    assert st.spot_checks >= st.fallback_spot + 1
