"""GPU parity of the single-species reaction-diffusion step (evx_rd_step) against the FP64
oracle, through the C ABI.  Tolerances as for the Cahn-Hilliard step: relative L2 over all
voxels, 1e-5 after one step and 1e-4 after twenty; closed forms (uniform map, linear-reaction
mode factor) to FP32 round-off."""
import os

import numpy as np
import pytest
import torch

from oracle import ch, reaction_diffusion as rd
from paper_2507_21748_amd.inputs import mode_field, quench_field

pytestmark = pytest.mark.gpu

ch.WORKERS = min(16, os.cpu_count() or 1)

SHAPES = [
    ((32, 32, 32), "periodic", "spectral"),
    ((32, 32, 32), "zero_flux", "stencil7"),
    ((40, 48, 24), "periodic", "stencil7"),
    ((24, 20, 100), "zero_flux", "spectral"),
    ((12, 96, 200), "periodic", "spectral"),
    ((48, 40, 512), "zero_flux", "stencil7"),
]


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_rd(evx, c0, bc, scheme, nsteps, p):
    plan = evx.Plan(c0.shape, bc, scheme, dx=p.dx)
    c = torch.from_numpy(np.ascontiguousarray(c0, dtype=np.float32)).cuda()
    plan.rd_step(c, nsteps, evx.RDParams(dt=p.dt, D=p.D, A=p.A, a0=p.a0, a1=p.a1, a2=p.a2,
                                         a3=p.a3))
    torch.cuda.synchronize()
    return c.cpu().numpy()


@pytest.mark.parametrize("shape,bc,scheme", SHAPES)
def test_rd_parity(evx_gpu, shape, bc, scheme):
    print(f"rd parity {shape} {bc} {scheme}", flush=True)
    p = rd.RDParams(dt=0.5, D=0.8, A=0.5, a0=0.05, a1=0.9, a2=-0.6, a3=-0.8)
    c0 = quench_field(shape, 0.3, 0.3, seed=41)
    one = gpu_rd(evx_gpu, c0, bc, scheme, 1, p)
    assert rel_l2(one, rd.rd_step(c0.astype(np.float64), p, bc, scheme)) <= 1e-5
    twenty = gpu_rd(evx_gpu, c0, bc, scheme, 20, p)
    assert rel_l2(twenty, rd.rd_run(c0, 20, p, bc, scheme)) <= 1e-4


def test_rd_logistic_front(evx_gpu):
    """Logistic growth (Fisher-KPP) from a seeded field, A = 0: the appendix's increment form."""
    shape = (64, 64, 64)
    p = rd.RDParams(dt=0.5, D=1.0, A=0.0, a0=0.0, a1=1.0, a2=-1.0, a3=0.0)
    c0 = np.clip(quench_field(shape, 0.0, 0.1, seed=42), 0.0, None).astype(np.float32)
    got = gpu_rd(evx_gpu, c0, "periodic", "spectral", 30, p)
    assert rel_l2(got, rd.rd_run(c0, 30, p, "periodic", "spectral")) <= 1e-4
    assert got.min() > -1e-3 and got.max() < 1.0 + 1e-3


def test_rd_uniform_map_and_linear_modes(evx_gpu):
    p = rd.RDParams(dt=0.7, D=0.6, A=1.0, a0=0.1, a1=-0.3, a2=0.8, a3=-0.5)
    c = np.full((16, 24, 32), 0.4, np.float32)
    got = gpu_rd(evx_gpu, c, "periodic", "spectral", 1, p)
    f = 0.1 - 0.3 * 0.4 + 0.8 * 0.16 - 0.5 * 0.064
    assert np.max(np.abs(got - (0.4 + p.dt * f / (1 + p.A * p.dt)))) <= 2e-7
    lin = rd.RDParams(dt=0.5, D=0.8, A=1.0, a0=0.0, a1=-0.3, a2=0.0, a3=0.0)
    shape, m, n = (16, 24, 32), (1, 2, 3), 10
    for bc in ("periodic", "zero_flux"):
        mode = mode_field(shape, 0.0, 1.0, m, bc).astype(np.float64)
        got = gpu_rd(evx_gpu, (0.7 * mode).astype(np.float32), bc, "stencil7", n, lin)
        K2 = sum(ch.axis_k2(s, lin.dx, bc, "stencil7")[mi] for s, mi in zip(shape, m))
        amp = np.sum(got * mode) / np.sum(mode * mode)
        assert abs(amp / (0.7 * rd.rd_growth_factor(K2, lin) ** n) - 1) <= 1e-5


def test_rd_dirichlet_needs_odd_reaction(evx_gpu):
    shape = (16, 24, 32)
    odd = rd.RDParams(dt=0.5, D=0.8, A=0.5, a0=0.0, a1=0.9, a2=0.0, a3=-0.8)
    c0 = quench_field(shape, 0.1, 0.3, seed=43)
    got = gpu_rd(evx_gpu, c0, "dirichlet", "stencil7", 5, odd)
    assert rel_l2(got, rd.rd_run(c0, 5, odd, "dirichlet", "stencil7")) <= 1e-5
    even = rd.RDParams(dt=0.5, a0=0.1)
    with pytest.raises(evx_gpu.EvxError) as ei:
        gpu_rd(evx_gpu, c0, "dirichlet", "stencil7", 1, even)
    assert ei.value.status == 3


def test_rd_leaves_no_cahn_hilliard_state(evx_gpu):
    """The step runs on the plan's buffers; a Cahn-Hilliard advance afterwards needs a begin."""
    shape = (16, 16, 16)
    plan = evx_gpu.Plan(shape, "periodic", "spectral")
    c = torch.from_numpy(quench_field(shape, 0.0, 0.1, seed=44)).cuda()
    plan.begin(c)
    plan.rd_step(c, 2, evx_gpu.RDParams())
    with pytest.raises(evx_gpu.EvxError) as ei:
        plan.advance(1, evx_gpu.CHParams(dt=0.5))
    assert ei.value.status == 6
