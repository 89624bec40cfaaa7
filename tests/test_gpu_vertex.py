"""GPU parity of vertex-centred zero-flux grids (n points j dx including both boundary vertices,
the field mirrored about them; DCT-I) against the FP64 oracle, through the C ABI.  The library
runs such an axis as the periodic transform of the even extension (length 2(n - 1)), reading it
mirrored and storing it cut.  Tolerances as for the other grids: relative L2 over all voxels,
1e-5 after one step and 1e-4 after twenty."""
import os

import numpy as np
import pytest
import torch

from oracle import ch
from oracle.ch import CHParams as OParams
from paper_2507_21748_amd.inputs import mode_field, quench_field
from tests.test_gpu_ch import gpu_run, rel_l2

pytestmark = pytest.mark.gpu

ch.WORKERS = min(16, os.cpu_count() or 1)
VX = "zero_flux_vertex"

CASES = [
    ((33, 33, 33), VX, "spectral"),
    ((33, 33, 33), VX, "stencil7"),
    ((65, 129, 33), VX, "stencil7"),
    ((16, 513, 32), ("periodic", VX, "periodic"), "spectral"),   # 1024-point extension along y
    ((16, 24, 513), ("zero_flux", "periodic", VX), "spectral"),  # 512-point x transform
    ((257, 20, 24), (VX, "dirichlet", "zero_flux"), "stencil7"),  # 512-point z extension
    ((21, 40, 41), (VX, "zero_flux", VX), "spectral"),            # radix-5 extensions (40, 80)
]


@pytest.mark.parametrize("shape,bc,scheme", CASES)
def test_vertex_parity(evx_gpu, shape, bc, scheme):
    print(f"vertex parity {shape} {bc} {scheme}", flush=True)
    p = OParams(dt=0.5, M=0.9, kappa=1.1, A=2.0)
    c0 = quench_field(shape, 0.1, 0.3, seed=81)
    one = gpu_run(evx_gpu, c0, bc, scheme, 1, p)
    assert rel_l2(one, ch.ch_step(c0.astype(np.float64), p, bc, scheme)) <= 1e-5
    twenty = gpu_run(evx_gpu, c0, bc, scheme, 20, p)
    assert rel_l2(twenty, ch.ch_run(c0, 20, p, bc, scheme)) <= 1e-4


def test_vertex_extension_identity_on_gpu(evx_gpu):
    """33 x 65 x 33 vertex grid for 5 steps = the periodic 64 x 128 x 64 step of its even
    extension (both on the GPU)."""
    p = OParams(dt=0.5)
    shape = (33, 65, 33)
    c0 = quench_field(shape, 0.0, 0.3, seed=82)
    e = c0
    for ax, n in enumerate(shape):
        e = np.concatenate([e, np.take(e, np.arange(n - 2, 0, -1), axis=ax)], axis=ax)
    per = gpu_run(evx_gpu, e.astype(np.float32), "periodic", "spectral", 5, p)[:33, :65, :33]
    got = gpu_run(evx_gpu, c0, VX, "spectral", 5, p)
    assert rel_l2(got, per) <= 2e-5


def test_vertex_cosine_mode_growth(evx_gpu):
    p = OParams(dt=0.5)
    shape, m, n, delta, cbar = (33, 65, 129), (1, 2, 3), 10, 1e-4, 0.1
    c0 = mode_field(shape, cbar, delta, m, VX)
    got = gpu_run(evx_gpu, c0, VX, "stencil7", n, p).astype(np.float64)
    mode = mode_field(shape, 0.0, 1.0, m, VX).astype(np.float64)
    K2 = sum(ch.axis_k2(s, p.dx, VX, "stencil7")[mi] for s, mi in zip(shape, m))
    amp = np.sum((got - np.mean(got)) * mode) / np.sum(mode * mode)
    a0 = np.sum((c0.astype(np.float64) - np.mean(c0)) * mode) / np.sum(mode * mode)
    assert abs(amp / (a0 * ch.growth_factor(K2, cbar, p) ** n) - 1) <= 2e-3


def test_vertex_reaction_diffusion_and_gray_scott(evx_gpu):
    from oracle import gray_scott as gs, reaction_diffusion as rd
    shape, bc = (17, 32, 65), (VX, "zero_flux", VX)
    p = rd.RDParams(dt=0.5, D=0.8, A=0.5, a0=0.05, a1=0.9, a2=-0.6, a3=-0.8)
    c0 = quench_field(shape, 0.3, 0.3, seed=83)
    plan = evx_gpu.Plan(shape, bc, "stencil7")
    c = torch.from_numpy(c0).cuda()
    plan.rd_step(c, 10, evx_gpu.RDParams(dt=p.dt, D=p.D, A=p.A, a0=p.a0, a1=p.a1, a2=p.a2,
                                         a3=p.a3))
    torch.cuda.synchronize()
    assert rel_l2(c.cpu().numpy(), rd.rd_run(c0, 10, p, bc, "stencil7")) <= 1e-4
    q = gs.GSParams(dt=0.8)
    u0 = quench_field(shape, 0.7, 0.3, seed=84)
    v0 = quench_field(shape, 0.2, 0.2, seed=85)
    plan = evx_gpu.Plan(shape, bc, "spectral", ops=evx_gpu.OP_GRAY_SCOTT)
    u, v = torch.from_numpy(u0).cuda(), torch.from_numpy(v0).cuda()
    plan.gs_step(u, v, 5, evx_gpu.GSParams(dt=q.dt, Du=q.Du, Dv=q.Dv, F=q.F, k=q.k))
    torch.cuda.synchronize()
    ur, vr = gs.gs_run(u0, v0, 5, q, bc, "spectral")
    assert rel_l2(u.cpu().numpy(), ur) <= 1e-4 and rel_l2(v.cpu().numpy(), vr) <= 1e-4


def test_vertex_refusals_and_sizes(evx_gpu):
    shape = (17, 17, 17)
    plan = evx_gpu.Plan(shape, VX, "spectral", ops=evx_gpu.OP_ADJOINT)
    c = torch.from_numpy(quench_field(shape, 0.0, 0.1, seed=86)).cuda()
    with pytest.raises(evx_gpu.EvxError) as ei:
        plan.diagnostics(c, evx_gpu.CHParams())
    assert ei.value.status == 3
    lam = c.clone()
    dk = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(evx_gpu.EvxError) as ei:
        plan.adjoint_step(c, lam, evx_gpu.CHParams(dt=0.5), dk, dk.clone())
    assert ei.value.status == 3
    with pytest.raises(evx_gpu.EvxError) as ei:
        evx_gpu.Plan((16, 16, 16), VX, "spectral")   # 2 (16 - 1) = 30 is not a supported length
    assert ei.value.status == 2
