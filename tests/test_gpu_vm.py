"""GPU parity of the variable-mobility Cahn-Hilliard step against the oracle through the C ABI:
1e-5 for one step and 1e-4 for 20 steps on several grids and boundaries (and the one-step
increment itself within 1e-4), mass conservation, uniform fields as exact fixed points, the
Dirichlet refusal and the workspace check."""
import os

import numpy as np
import pytest
import torch

from oracle import ch, ch_varmob as vm
from paper_2507_21748_amd.inputs import quench_field

pytestmark = pytest.mark.gpu

ch.WORKERS = min(16, os.cpu_count() or 1)


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_vm(evx, phi0, bc, scheme, nsteps, p):
    plan = evx.Plan(phi0.shape, bc, scheme, dx=p.dx, ops=evx.OP_STEP | evx.OP_VAR_MOBILITY)
    phi = torch.from_numpy(np.ascontiguousarray(phi0, dtype=np.float32)).cuda()
    plan.vm_step(phi, nsteps, evx.VMParams(dt=p.dt, D0=p.D0, gamma0=p.gamma0, eps=p.eps,
                                           M0=p.M0))
    torch.cuda.synchronize()
    return phi.cpu().numpy()


SHAPES = [
    ((32, 32, 32), "periodic", "spectral"),
    ((32, 32, 32), "zero_flux", "stencil7"),
    ((40, 48, 24), "periodic", "stencil7"),
    ((24, 20, 100), "zero_flux", "spectral"),
    ((24, 20, 32), ("zero_flux", "periodic", "periodic"), "spectral"),
]

P = vm.VMParams(dx=1.0, dt=0.5, D0=1.2, gamma0=0.9, eps=1.8, M0=0.3)


@pytest.mark.parametrize("shape,bc,scheme", SHAPES)
def test_one_and_twenty_steps(evx_gpu, shape, bc, scheme):
    phi0 = quench_field(shape, 0.5, 0.2, seed=81)
    one = gpu_vm(evx_gpu, phi0, bc, scheme, 1, P)
    ref = vm.vm_step(phi0.astype(np.float64), P, bc, scheme)
    assert rel_l2(one, ref) <= 1e-5
    assert rel_l2(one - phi0, ref - phi0) <= 1e-4
    twenty = gpu_vm(evx_gpu, phi0, bc, scheme, 20, P)
    ref = vm.vm_run(phi0, 20, P, bc, scheme)
    assert rel_l2(twenty, ref) <= 1e-4
    assert abs(float(np.mean(twenty, dtype=np.float64)) - float(np.mean(phi0, dtype=np.float64))) < 1e-6


@pytest.mark.parametrize("bc,scheme", [("periodic", "spectral"), ("zero_flux", "stencil7")])
def test_full_size_against_oracle(evx_gpu, bc, scheme):
    """128^3, two steps, every voxel against the oracle."""
    shape = (128, 128, 128)
    phi0 = quench_field(shape, 0.5, 0.2, seed=82)
    out = gpu_vm(evx_gpu, phi0, bc, scheme, 2, P)
    ref = vm.vm_run(phi0, 2, P, bc, scheme)
    assert rel_l2(out, ref) <= 1e-5
    assert np.max(np.abs(out - ref)) <= 1e-4


def test_uniform_fields_are_fixed_points(evx_gpu):
    for v in (0.0, 0.3, 1.0):
        phi = gpu_vm(evx_gpu, np.full((16, 16, 16), v, np.float32), "zero_flux", "stencil7", 5, P)
        assert np.array_equal(phi, np.full((16, 16, 16), v, np.float32))


def test_dirichlet_refused_and_workspace_required(evx_gpu):
    phi = torch.full((16, 16, 16), 0.5, device="cuda")
    plan = evx_gpu.Plan((16, 16, 16), "dirichlet", "spectral",
                        ops=evx_gpu.OP_STEP | evx_gpu.OP_VAR_MOBILITY)
    with pytest.raises(evx_gpu.EvxError) as e:
        plan.vm_step(phi, 1, evx_gpu.VMParams())
    assert e.value.status == 3  # EVX_ERR_UNSUPPORTED
    plan = evx_gpu.Plan((16, 16, 16), "periodic", "spectral")
    with pytest.raises(evx_gpu.EvxError) as e:
        plan.vm_step(phi, 1, evx_gpu.VMParams())
    assert e.value.status == 4  # EVX_ERR_NOMEM
