"""GPU parity of the Gray-Scott two-species model against the oracle through the C ABI: 1e-5 for
one step and 1e-4 for 20 steps on several grids and boundaries, the uniform reaction map, and
the fixed point (1, 0)."""
import os

import numpy as np
import pytest
import torch

from oracle import ch, gray_scott as gs
from paper_2507_21748_amd.inputs import quench_field

pytestmark = pytest.mark.gpu

ch.WORKERS = min(16, os.cpu_count() or 1)


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_gs(evx, u0, v0, bc, scheme, nsteps, p):
    plan = evx.Plan(u0.shape, bc, scheme, dx=p.dx, ops=evx.OP_STEP | evx.OP_GRAY_SCOTT)
    u = torch.from_numpy(np.ascontiguousarray(u0, dtype=np.float32)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(v0, dtype=np.float32)).cuda()
    plan.gs_step(u, v, nsteps, evx.GSParams(dt=p.dt, Du=p.Du, Dv=p.Dv, F=p.F, k=p.k))
    torch.cuda.synchronize()
    return u.cpu().numpy(), v.cpu().numpy()


SHAPES = [
    ((32, 32, 32), "periodic", "spectral"),
    ((32, 32, 32), "zero_flux", "stencil7"),
    ((40, 48, 24), "periodic", "stencil7"),
    ((24, 20, 100), "zero_flux", "spectral"),
    ((24, 20, 32), ("dirichlet", "zero_flux", "periodic"), "spectral"),
]


@pytest.mark.parametrize("shape,bc,scheme", SHAPES)
def test_one_and_twenty_steps(evx_gpu, shape, bc, scheme):
    p = gs.GSParams(dt=0.8)
    u0 = quench_field(shape, 0.7, 0.3, seed=71)
    v0 = quench_field(shape, 0.2, 0.2, seed=72)
    u1, v1 = gpu_gs(evx_gpu, u0, v0, bc, scheme, 1, p)
    ur, vr = gs.gs_step(u0, v0, p, bc, scheme)
    assert rel_l2(u1, ur) <= 1e-5 and rel_l2(v1, vr) <= 1e-5
    u20, v20 = gpu_gs(evx_gpu, u0, v0, bc, scheme, 20, p)
    ur, vr = gs.gs_run(u0, v0, 20, p, bc, scheme)
    assert rel_l2(u20, ur) <= 1e-4 and rel_l2(v20, vr) <= 1e-4


def test_uniform_map_and_fixed_point(evx_gpu):
    p = gs.GSParams(dt=0.7)
    shape = (16, 16, 16)
    u, v = gpu_gs(evx_gpu, np.full(shape, 0.5), np.full(shape, 0.25), "periodic", "spectral", 1, p)
    uv2 = 0.5 * 0.25 * 0.25
    assert np.max(np.abs(u - (0.5 + p.dt * (-uv2 + p.F * 0.5)))) < 1e-6
    assert np.max(np.abs(v - (0.25 + p.dt * (uv2 - p.k * 0.25)))) < 1e-6
    u, v = gpu_gs(evx_gpu, np.ones(shape), np.zeros(shape), "zero_flux", "stencil7", 10, p)
    assert np.max(np.abs(u - 1.0)) < 1e-6 and np.max(np.abs(v)) < 1e-6


def test_workspace_required(evx_gpu):
    plan = evx_gpu.Plan((16, 16, 16), "periodic", "spectral")
    u = torch.ones((16, 16, 16), device="cuda")
    v = torch.zeros((16, 16, 16), device="cuda")
    with pytest.raises(evx_gpu.EvxError) as e:
        plan.gs_step(u, v, 1, evx_gpu.GSParams())
    assert e.value.status == 4  # EVX_ERR_NOMEM
