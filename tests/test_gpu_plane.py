"""The plane pass (one launch per z plane running the inverse y, fused x and forward y transforms
on the plane's spectrum held in LDS; periodic grids with nx = ny = 32 or 64) against the three
separate passes (bitwise: the same FFT plans, tables and operation order) and against the FP64
oracle (relative L2 over all voxels: 1e-5 after one step, 1e-4 after ten)."""
import os

import numpy as np
import pytest
import torch

from oracle import ch
from oracle.ch import CHParams as OParams
from paper_2507_21748_amd.inputs import quench_field

pytestmark = pytest.mark.gpu

ch.WORKERS = min(16, os.cpu_count() or 1)


def _run(evx, shape, scheme, prm, nsteps, plane, seed=95):
    plan = evx.Plan(shape, "periodic", scheme)
    plan.set_plane_pass(plane)
    c = torch.from_numpy(quench_field(shape, 0.05, 0.3, seed=seed)).cuda()
    plan.step(c, nsteps, prm)
    torch.cuda.synchronize()
    return c.cpu().numpy()


@pytest.mark.parametrize("shape,scheme", [((64, 64, 64), "spectral"),
                                          ((40, 32, 32), "stencil7"),
                                          ((32, 32, 32), "spectral"),
                                          ((20, 64, 64), "stencil7")])
@pytest.mark.parametrize("integrator,model", [(0, 0), (1, 0), (0, 1)])
def test_plane_pass_is_bitwise_the_three_passes(evx_gpu, shape, scheme, integrator, model):
    print(f"plane pass {shape} {scheme} integrator {integrator} model {model}", flush=True)
    prm = evx_gpu.CHParams(dt=0.5, M=0.9, kappa=1.1, integrator=integrator, model=model)
    a = _run(evx_gpu, shape, scheme, prm, 7, True)
    b = _run(evx_gpu, shape, scheme, prm, 7, False)
    assert np.isfinite(a).all()
    assert np.array_equal(a, b), float(np.max(np.abs(a - b)))


@pytest.mark.parametrize("shape,scheme", [((24, 64, 64), "spectral"), ((16, 32, 32), "stencil7")])
def test_plane_pass_matches_oracle(evx_gpu, shape, scheme):
    p = OParams(dt=0.5, M=0.9, kappa=1.1, A=2.0)
    prm = evx_gpu.CHParams(dt=p.dt, M=p.M, kappa=p.kappa, A=p.A)
    c0 = quench_field(shape, 0.05, 0.3, seed=95)
    one = _run(evx_gpu, shape, scheme, prm, 1, True)
    ref = ch.ch_step(c0.astype(np.float64), p, "periodic", scheme)
    assert np.linalg.norm(one - ref) / np.linalg.norm(ref) <= 1e-5
    ten = _run(evx_gpu, shape, scheme, prm, 10, True)
    ref = ch.ch_run(c0, 10, p, "periodic", scheme)
    assert np.linalg.norm(ten - ref) / np.linalg.norm(ref) <= 1e-4


def test_plane_pass_with_graph_replay_and_other_grids(evx_gpu):
    """Captured steps replay the plane pass (bitwise equal to eager three-pass steps); on grids
    the plane pass does not cover, switching it changes nothing."""
    shape = (64, 64, 64)
    prm = evx_gpu.CHParams(dt=0.5)
    plan = evx_gpu.Plan(shape, "periodic", "spectral")
    plan.set_step_graph(8)
    c = torch.from_numpy(quench_field(shape, 0.05, 0.3, seed=96)).cuda()  # as _run draws it
    plan.step(c, 24, prm)
    ref = _run(evx_gpu, shape, "spectral", prm, 24, False, seed=96)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), ref)
    for shape2, bc in [((32, 48, 64), "periodic"), ((16, 64, 64), "zero_flux"),
                       ((16, 128, 128), "periodic")]:
        outs = []
        for on in (True, False):
            plan = evx_gpu.Plan(shape2, bc, "spectral")
            plan.set_plane_pass(on)
            c = torch.from_numpy(quench_field(shape2, 0.0, 0.3, seed=97)).cuda()
            plan.step(c, 3, prm)
            torch.cuda.synchronize()
            outs.append(c.cpu().numpy())
        assert np.array_equal(outs[0], outs[1])
