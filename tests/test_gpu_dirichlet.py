"""GPU parity of Dirichlet grids (zero-flux kernels on the sign-alternated field, reversed K2)
against the oracle's DST-II steps through the C ABI (1e-5 for one step, 1e-4 for 20 steps), the
odd-extension identity with the GPU's own periodic step at a size the oracle does not step, sine
mode growth, and the diagnostics."""
import os

import numpy as np
import pytest
import torch

from oracle import ch
from oracle.ch import CHParams as OParams
from paper_2507_21748_amd.inputs import quench_field

pytestmark = pytest.mark.gpu

ch.WORKERS = min(16, os.cpu_count() or 1)


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_run(evx, c0, bc, scheme, nsteps, p: OParams):
    plan = evx.Plan(c0.shape, bc, scheme, dx=p.dx)
    c = torch.from_numpy(np.ascontiguousarray(c0, dtype=np.float32)).cuda()
    plan.step(c, nsteps, evx.CHParams(dt=p.dt, M=p.M, kappa=p.kappa, A=p.A))
    torch.cuda.synchronize()
    return c.cpu().numpy()


SHAPES = [
    ((32, 32, 32), "spectral"),
    ((32, 32, 32), "stencil7"),
    ((40, 48, 24), "stencil7"),
    ((24, 20, 100), "spectral"),
    ((12, 96, 200), "spectral"),
    ((50, 40, 48), "stencil7"),
]


@pytest.mark.parametrize("shape,scheme", SHAPES)
def test_one_step_parity(evx_gpu, shape, scheme):
    p = OParams(dt=0.5)
    c0 = quench_field(shape, 0.1, 0.3, seed=61)
    got = gpu_run(evx_gpu, c0, "dirichlet", scheme, 1, p)
    ref = ch.ch_step(c0.astype(np.float64), p, "dirichlet", scheme)
    assert rel_l2(got, ref) <= 1e-5


@pytest.mark.parametrize("shape,scheme", SHAPES[:4])
def test_twenty_step_parity(evx_gpu, shape, scheme):
    p = OParams(dt=0.5, M=0.8, kappa=1.3, A=2.0)
    c0 = quench_field(shape, 0.0, 0.3, seed=62)
    got = gpu_run(evx_gpu, c0, "dirichlet", scheme, 20, p)
    ref = ch.ch_run(c0, 20, p, "dirichlet", scheme)
    assert rel_l2(got, ref) <= 1e-4


@pytest.mark.parametrize("scheme", ["spectral", "stencil7"])
def test_odd_extension_identity_256(evx_gpu, scheme):
    """Dirichlet 128 x 64 x 128 for 5 steps = periodic 256 x 128 x 256 on the odd extension about
    the cell faces, restricted (both on the GPU)."""
    p = OParams(dt=0.5)
    c0 = quench_field((128, 64, 128), 0.0, 0.3, seed=63)
    e = c0
    for ax in range(3):
        e = np.concatenate([e, -np.flip(e, axis=ax)], axis=ax)
    per = gpu_run(evx_gpu, e, "periodic", scheme, 5, p)[:128, :64, :128]
    d = gpu_run(evx_gpu, c0, "dirichlet", scheme, 5, p)
    assert rel_l2(d, per) <= 2e-5


def test_sine_mode_growth(evx_gpu):
    p = OParams(dt=0.5)
    shape, m, n, delta = (24, 40, 48), (1, 2, 3), 10, 1e-4
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    mode = np.ones(shape)
    for g, s, mi in zip(grids, shape, m):
        mode = mode * np.sin(np.pi * mi * (g + 0.5) / s)
    got = gpu_run(evx_gpu, (delta * mode).astype(np.float32), "dirichlet", "spectral", n, p)
    amp = np.sum(got.astype(np.float64) * mode) / np.sum(mode * mode)
    K2 = sum(ch.axis_k2(s, p.dx, "dirichlet", "spectral")[mi - 1] for s, mi in zip(shape, m))
    assert abs(amp / (delta * ch.growth_factor(K2, 0.0, p) ** n) - 1.0) <= 2e-3


@pytest.mark.parametrize("scheme", ["spectral", "stencil7"])
def test_diagnostics(evx_gpu, scheme):
    """Mass (real-space sum) and energy (Parseval sum with the reversed K2) against the oracle."""
    shape = (24, 20, 32)
    p = OParams(dt=0.5, kappa=1.2)
    c0 = quench_field(shape, 0.1, 0.4, seed=64)
    plan = evx_gpu.Plan(shape, "dirichlet", scheme, ops=evx_gpu.OP_STEP | evx_gpu.OP_DIAG)
    c = torch.from_numpy(c0).cuda()
    mass, energy = plan.diagnostics(c, evx_gpu.CHParams(dt=p.dt, kappa=p.kappa)).tolist()
    c64 = c0.astype(np.float64)
    assert abs(mass / ch.mass(c64, p.dx) - 1.0) <= 1e-5
    assert abs(energy / ch.energy(c64, p, "dirichlet", scheme) - 1.0) <= 1e-5


@pytest.mark.parametrize("which", ["etd1", "allen_cahn", "allen_cahn_etd1"])
def test_with_other_integrators_and_models(evx_gpu, which):
    """Dirichlet grids with the exponential integrator and the Allen-Cahn model: one step against
    the oracle's DST-II versions of those steps."""
    shape, scheme = (24, 20, 32), "stencil7"
    p = OParams(dt=0.5, M=0.9, kappa=1.1, A=2.0)
    c0 = quench_field(shape, 0.1, 0.3, seed=65)
    etd1 = which.endswith("etd1")
    ac = which.startswith("allen")
    plan = evx_gpu.Plan(shape, "dirichlet", scheme)
    c = torch.from_numpy(c0).cuda()
    plan.step(c, 1, evx_gpu.CHParams(dt=p.dt, M=p.M, kappa=p.kappa, A=p.A,
                                     integrator=evx_gpu.ETD1 if etd1 else evx_gpu.SEMI_IMPLICIT,
                                     model=evx_gpu.ALLEN_CAHN if ac else evx_gpu.CAHN_HILLIARD))
    torch.cuda.synchronize()
    c64 = c0.astype(np.float64)
    if ac:
        ref = ch.ac_run(c64, 1, p, "dirichlet", scheme, etd1=etd1)
    else:
        ref = ch.ch_step_etd1(c64, p, "dirichlet", scheme)
    assert rel_l2(c.cpu().numpy(), ref) <= 1e-5


MIXES = [("dirichlet", "zero_flux", "zero_flux"), ("zero_flux", "dirichlet", "dirichlet"),
         ("zero_flux", "zero_flux", "dirichlet"), ("zero_flux", "dirichlet", "periodic"),
         ("periodic", "zero_flux", "periodic"), ("dirichlet", "periodic", "periodic"),
         # a periodic y or z under a cosine x: one complex column per x bin
         ("periodic", "zero_flux", "dirichlet"), ("zero_flux", "periodic", "zero_flux"),
         ("periodic", "periodic", "zero_flux")]


@pytest.mark.parametrize("bcs", MIXES)
@pytest.mark.parametrize("scheme", ["spectral", "stencil7"])
def test_mixed_axes_parity(evx_gpu, bcs, scheme):
    """Per-axis boundaries (z, y, x): one step within 1e-5 and 20 steps within 1e-4 of the
    oracle."""
    shape = (24, 20, 32)
    p = OParams(dt=0.5, M=0.8, kappa=1.3, A=2.0)
    c0 = quench_field(shape, 0.0, 0.3, seed=66)
    got1 = gpu_run(evx_gpu, c0, bcs, scheme, 1, p)
    assert rel_l2(got1, ch.ch_step(c0.astype(np.float64), p, bcs, scheme)) <= 1e-5
    got20 = gpu_run(evx_gpu, c0, bcs, scheme, 20, p)
    assert rel_l2(got20, ch.ch_run(c0, 20, p, bcs, scheme)) <= 1e-4


def test_mixed_axes_extension_identity_on_gpu(evx_gpu):
    """z Dirichlet, y zero flux, x Dirichlet at 64 x 96 x 128 for 5 steps = periodic
    128 x 192 x 256 on the extension odd in z and x and even in y (both on the GPU)."""
    p = OParams(dt=0.5)
    bcs = ("dirichlet", "zero_flux", "dirichlet")
    c0 = quench_field((64, 96, 128), 0.0, 0.3, seed=67)
    e = c0
    for ax, b in enumerate(bcs):
        e = np.concatenate([e, (-1.0 if b == "dirichlet" else 1.0) * np.flip(e, axis=ax)], axis=ax)
    per = gpu_run(evx_gpu, e.astype(np.float32), "periodic", "spectral", 5, p)[:64, :96, :128]
    got = gpu_run(evx_gpu, c0, bcs, "spectral", 5, p)
    assert rel_l2(got, per) <= 2e-5


def test_periodic_yz_under_cosine_x_extension_identity_on_gpu(evx_gpu):
    """z periodic, y zero flux, x Dirichlet at 64 x 48 x 96 for 5 steps = periodic
    64 x 96 x 192 on the extension even in y and odd in x (both on the GPU)."""
    p = OParams(dt=0.5)
    bcs = ("periodic", "zero_flux", "dirichlet")
    c0 = quench_field((64, 48, 96), 0.0, 0.3, seed=68)
    e = c0
    for ax, b in enumerate(bcs):
        if b != "periodic":
            e = np.concatenate([e, (-1.0 if b == "dirichlet" else 1.0) * np.flip(e, axis=ax)],
                               axis=ax)
    per = gpu_run(evx_gpu, e.astype(np.float32), "periodic", "spectral", 5, p)[:64, :48, :96]
    got = gpu_run(evx_gpu, c0, bcs, "spectral", 5, p)
    assert rel_l2(got, per) <= 2e-5


@pytest.mark.parametrize("bcs", [("periodic", "zero_flux", "zero_flux"),
                                 ("zero_flux", "periodic", "dirichlet")])
def test_periodic_yz_under_cosine_x_diagnostics_and_adjoint(evx_gpu, bcs):
    """Mass, energy and one adjoint step on the complex-column layout against the oracle."""
    from oracle import adjoint as oadj
    shape = (16, 24, 32)
    p = OParams(dt=0.5, M=0.8, kappa=1.3, A=2.0)
    c0 = quench_field(shape, 0.1, 0.3, seed=69)
    plan = evx_gpu.Plan(shape, bcs, "stencil7", ops=evx_gpu.OP_ADJOINT)
    c = torch.from_numpy(c0).cuda()
    d = plan.diagnostics(c, evx_gpu.CHParams(dt=p.dt, M=p.M, kappa=p.kappa, A=p.A)).cpu().numpy()
    c64 = c0.astype(np.float64)
    assert abs(d[0] - ch.mass(c64)) <= 1e-6 * np.sum(np.abs(c64))
    assert abs(d[1] / ch.energy(c64, p, bcs, "stencil7") - 1) <= 1e-6
    lam0 = quench_field(shape, 0.0, 1.0, seed=70)
    c1 = ch.ch_step(c64, p, bcs, "stencil7")
    target = c1 - lam0.astype(np.float64) / 2          # so that dL/dc^1 = lam0
    _, ref_lam, ref_dk, ref_dM = oadj.adjoint_gradients(c0, target, 1, p, bcs, "stencil7")
    lam = torch.from_numpy(lam0).cuda()
    dk = torch.zeros(1, dtype=torch.float64, device="cuda")
    dM = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.adjoint_step(c, lam, evx_gpu.CHParams(dt=p.dt, M=p.M, kappa=p.kappa, A=p.A), dk, dM)
    torch.cuda.synchronize()
    assert rel_l2(lam.cpu().numpy(), ref_lam) <= 1e-5
    assert abs(dk.item() / ref_dk - 1) <= 1e-5 and abs(dM.item() / ref_dM - 1) <= 1e-5
