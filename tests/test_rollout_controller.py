"""The coarse-stepper rollout controller's decisions, driven on the CPU by a fake solver built on
the FP64 oracle and by mock networks (no GPU): an exact network is always accepted, a
mass-violating one falls back on mass, an energy-raising one on energy, and a slightly wrong one
is caught by the spot check; every fallback replaces the prediction by the solver's steps."""
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
        return out


def _run(kind, napps=6):
    shape = (12, 12, 12)
    plan = FakePlan(shape)
    c0 = torch.from_numpy(quench_field(shape, 0.0, 0.05, seed=1))
    cfg = RolloutConfig(check_every=2, conserve_mass=False)
    c, st = rollout(MockNet(plan, kind), c0, napps, evx.CHParams(dt=0.5), cfg, plan=plan)
    ref = c0.clone()
    plan.step(ref, 10 * napps, evx.CHParams(dt=0.5))
    return c, ref, st


def test_exact_network_always_accepted():
    c, ref, st = _run("exact")
    assert st.accepted == st.applications == 6 and st.spot_checks == 3
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
