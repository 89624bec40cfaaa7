"""GPU parity of the HIP spectral CH stepper against the FP64 oracle, through the C ABI.

Tolerances (relative L2 over all voxels, FP64 evaluation): 1e-5 for one step and 1e-3 after the
long runs, as the method's accuracy targets state; short multi-step runs get 1e-4.  Full-size
grids that the oracle cannot step in seconds are checked through properties that hold at any
size: periodic tiling and mirror tiling (the step of a repeated block is the repeated step of
the block), single-mode linear growth at an arbitrary bin, mass conservation and determinism.
"""
import os

import numpy as np
import pytest
import torch

from oracle import ch
from oracle.ch import CHParams as OParams
from paper_2507_21748_amd.inputs import mode_field, quench_field

pytestmark = pytest.mark.gpu

ch.WORKERS = min(16, os.cpu_count() or 1)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_run(evx, c0, bc, scheme, nsteps, p: OParams, remap=True):
    plan = evx.Plan(c0.shape, bc, scheme, dx=p.dx)
    plan.set_xcd_remap(remap)
    c = torch.from_numpy(np.ascontiguousarray(c0, dtype=np.float32)).cuda()
    plan.step(c, nsteps, evx.CHParams(dt=p.dt, M=p.M, kappa=p.kappa, A=p.A))
    torch.cuda.synchronize()
    return c.cpu().numpy()


SHAPES = [
    ((32, 32, 32), "periodic", "spectral"),
    ((32, 32, 32), "zero_flux", "stencil7"),
    ((40, 48, 24), "periodic", "stencil7"),
    ((24, 20, 100), "zero_flux", "spectral"),
    ((12, 96, 200), "periodic", "spectral"),
    ((50, 40, 48), "zero_flux", "stencil7"),
    ((64, 128, 80), "periodic", "spectral"),
    ((16, 8, 12), "zero_flux", "spectral"),
    ((4, 6, 8), "periodic", "spectral"),
    ((100, 64, 160), "zero_flux", "stencil7"),
    ((20, 384, 96), "periodic", "stencil7"),
    ((192, 10, 320), "zero_flux", "spectral"),
]


@pytest.mark.parametrize("shape,bc,scheme", SHAPES)
def test_one_step_parity(evx_gpu, shape, bc, scheme):
    p = OParams(dt=0.5)
    c0 = quench_field(shape, 0.1, 0.3, seed=21)
    got = gpu_run(evx_gpu, c0, bc, scheme, 1, p)
    ref = ch.ch_step(c0.astype(np.float64), p, bc, scheme)
    assert rel_l2(got, ref) <= 1e-5


@pytest.mark.parametrize("shape,bc,scheme", SHAPES[:6])
def test_twenty_step_parity(evx_gpu, shape, bc, scheme):
    p = OParams(dt=0.5, M=0.8, kappa=1.3, A=2.0)
    c0 = quench_field(shape, 0.0, 0.05, seed=22)
    got = gpu_run(evx_gpu, c0, bc, scheme, 20, p)
    ref = ch.ch_run(c0, 20, p, bc, scheme)
    assert rel_l2(got, ref) <= 1e-4


def test_small_quench_config(evx_gpu):
    """32^3 periodic spectral, mean 0, amplitude 0.05, seed 1, dt 0.1, 100 steps."""
    p = OParams(dt=0.1)
    c0 = quench_field((32, 32, 32), 0.0, 0.05, seed=1)
    one = gpu_run(evx_gpu, c0, "periodic", "spectral", 1, p)
    assert rel_l2(one, ch.ch_step(c0.astype(np.float64), p, "periodic", "spectral")) <= 1e-5
    got = gpu_run(evx_gpu, c0, "periodic", "spectral", 100, p)
    ref = ch.ch_run(c0, 100, p, "periodic", "spectral")
    err = rel_l2(got, ref)
    print(f"32^3 100 steps rel L2 = {err:.3e}")
    assert err <= 1e-3


def test_zero_steps_is_round_trip(evx_gpu):
    c0 = quench_field((24, 32, 40), 0.2, 0.5, seed=3)
    for bc in ("periodic", "zero_flux"):
        got = gpu_run(evx_gpu, c0, bc, "spectral", 0, OParams())
        assert np.max(np.abs(got - c0)) <= 2e-6


def test_constant_field_is_fixed_point(evx_gpu):
    for bc in ("periodic", "zero_flux"):
        c0 = np.full((16, 32, 64), 0.37, np.float32)
        got = gpu_run(evx_gpu, c0, bc, "stencil7", 10, OParams(dt=0.5))
        assert np.max(np.abs(got - 0.37)) <= 1e-6


@pytest.mark.parametrize("bc", ["periodic", "zero_flux"])
def test_mass_dc_bin_bit_exact(evx_gpu, bc):
    shape = (32, 40, 48)
    c0 = quench_field(shape, 0.2, 0.05, seed=4)
    plan = evx_gpu.Plan(shape, bc, "spectral")
    c = torch.from_numpy(c0).cuda()
    plan.begin(c)
    st = plan.state().view(torch.float32)
    dc0 = st[0].item()
    plan.advance(200, evx_gpu.CHParams(dt=0.5))
    torch.cuda.synchronize()
    assert st[0].item() == dc0
    plan.end(c)
    assert abs(float(c.double().mean()) - float(c0.astype(np.float64).mean())) <= 1e-6


@pytest.mark.parametrize("bc,scheme", [("periodic", "spectral"), ("zero_flux", "stencil7")])
def test_energy_monotone(evx_gpu, bc, scheme):
    p = OParams(dt=0.5)
    shape = (32, 32, 32)
    plan = evx_gpu.Plan(shape, bc, scheme)
    c = torch.from_numpy(quench_field(shape, 0.0, 0.05, seed=5)).cuda()
    prm = evx_gpu.CHParams(dt=0.5)
    plan.begin(c)
    E = []
    for _ in range(30):
        plan.end(c)
        E.append(ch.energy(c.cpu().numpy().astype(np.float64), p, bc, scheme))
        plan.advance(10, prm)
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-6 * np.abs(E[:-1]))
    assert E[-1] < 0.8 * E[0]


@pytest.mark.parametrize("shape,bc,scheme,m", [
    ((32, 32, 32), "periodic", "spectral", (1, 2, 3)),
    ((24, 40, 48), "zero_flux", "stencil7", (3, 1, 2)),
    ((24, 40, 48), "periodic", "stencil7", (2, 3, 1)),
])
@pytest.mark.parametrize("cbar", [0.0, 0.2])
def test_linear_growth(evx_gpu, shape, bc, scheme, m, cbar):
    """A mode of amplitude 1e-4 grows by the closed-form factor g(K2)^n."""
    p = OParams(dt=0.5)
    n, delta = 10, 1e-4
    mode = mode_field(shape, 0.0, 1.0, m, bc).astype(np.float64)
    c0 = (cbar + delta * mode).astype(np.float32)
    got = gpu_run(evx_gpu, c0, bc, scheme, n, p).astype(np.float64)
    amp = np.sum((got - got.mean()) * mode) / np.sum(mode * mode)
    amp0 = np.sum((c0 - c0.astype(np.float64).mean()) * mode) / np.sum(mode * mode)
    K2 = sum(ch.axis_k2(s, p.dx, bc, scheme)[mi] for s, mi in zip(shape, m))
    g = ch.growth_factor(K2, float(c0.astype(np.float64).mean()), p)
    assert abs(amp / (amp0 * g ** n) - 1.0) <= 2e-3


def test_resume_is_bitwise(evx_gpu):
    shape = (32, 24, 40)
    prm = evx_gpu.CHParams(dt=0.5)
    c0 = quench_field(shape, 0.1, 0.05, seed=7)
    plan = evx_gpu.Plan(shape, "periodic", "spectral")
    a = torch.from_numpy(c0).cuda()
    plan.begin(a)
    plan.advance(20, prm)
    saved = plan.state().clone()
    plan.advance(20, prm)
    plan.end(a)
    b = torch.empty_like(a)
    plan.state().copy_(saved)
    plan.restore()
    plan.advance(20, prm)
    plan.end(b)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_deterministic_and_remap_invariant(evx_gpu):
    c0 = quench_field((64, 64, 64), 0.0, 0.05, seed=8)
    p = OParams(dt=0.5)
    a = gpu_run(evx_gpu, c0, "periodic", "spectral", 30, p, remap=True)
    b = gpu_run(evx_gpu, c0, "periodic", "spectral", 30, p, remap=True)
    c = gpu_run(evx_gpu, c0, "periodic", "spectral", 30, p, remap=False)
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)


# ------------------------------------------------------------------ full-size grids
@pytest.mark.parametrize("bc,scheme", [("periodic", "spectral"), ("zero_flux", "stencil7")])
def test_256_parity(evx_gpu, bc, scheme):
    """256^3 off-critical quench (mean 0.2): 1 and 10 steps against the oracle run here."""
    p = OParams(dt=0.5)
    c0 = quench_field((256, 256, 256), 0.2, 0.05, seed=2)
    ref = c0.astype(np.float64)
    for n, tol in ((1, 1e-5), (9, 1e-4)):
        for _ in range(n):
            ref = ch.ch_step(ref, p, bc, scheme)
        got = gpu_run(evx_gpu, c0, bc, scheme, 1 if n == 1 else 10, p)
        assert rel_l2(got, ref) <= tol


@pytest.mark.parametrize("variant,bc,scheme", [("periodic", "periodic", "spectral"),
                                               ("zero_flux", "zero_flux", "stencil7")])
def test_256_thousand_steps_sampled(evx_gpu, variant, bc, scheme):
    """256^3, 1000 steps of dt 0.5, against stored oracle samples (tests/golden)."""
    path = os.path.join(GOLDEN, f"ch256_{variant}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    g = np.load(path, allow_pickle=False)
    idx = g["index"]
    p = OParams(dt=0.5)
    plan = evx_gpu.Plan((256, 256, 256), bc, scheme)
    c = torch.from_numpy(quench_field((256, 256, 256), 0.2, 0.05, seed=2)).cuda()
    prm = evx_gpu.CHParams(dt=p.dt)
    plan.begin(c)
    done = 0
    for n in g["steps"]:
        plan.advance(int(n) - done, prm)
        done = int(n)
        out = torch.empty_like(c)
        plan.end(out)
        got = out.cpu().numpy().reshape(-1)[idx].astype(np.float64)
        ref = g[f"values_{n}"]
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        print(f"{variant} step {n}: sampled rel L2 {err:.3e}")
        assert err <= (1e-5 if n == 1 else 1e-3)


def _tile_check(big, small_ref, reps):
    """max relative L2 over z-slabs of big vs np.tile(small_ref), evaluated slab-wise."""
    nz = small_ref.shape[0]
    num = den = 0.0
    row = np.tile(small_ref, (1, reps[1], reps[2]))
    for z0 in range(0, big.shape[0], nz):
        d = big[z0:z0 + nz].astype(np.float64) - row
        num += float(np.sum(d * d))
        den += float(np.sum(row * row))
    return (num / den) ** 0.5


def test_1024_periodic_tiled(evx_gpu):
    """1024^3 periodic spectral: a 32^3 block repeated 32 times per axis steps to the repeated
    oracle step of the block (every pass of the full-size launch is exercised)."""
    p = OParams(dt=0.5)
    small = quench_field((32, 32, 32), 0.0, 0.05, seed=3)
    big = np.tile(small, (32, 32, 32))
    ref = ch.ch_run(small, 5, p, "periodic", "spectral")
    got = gpu_run(evx_gpu, big, "periodic", "spectral", 5, p)
    del big
    assert _tile_check(got, ref, (32, 32, 32)) <= 1e-5


def test_1024_periodic_mode_growth_and_mass(evx_gpu):
    """1024^3: a single mode at a bin that is not a multiple of any tile grows by g^n."""
    p = OParams(dt=0.5)
    shape, m, n, delta = (1024, 1024, 1024), (3, 7, 11), 5, 1e-4
    iz = np.arange(1024)[:, None, None]
    iy = np.arange(1024)[None, :, None]
    ix = np.arange(1024)[None, None, :]
    c0 = np.empty(shape, np.float32)
    for z0 in range(0, 1024, 64):
        ph = 2 * np.pi * (m[2] * ix / 1024 + m[1] * iy / 1024 + m[0] * iz[z0:z0 + 64] / 1024)
        c0[z0:z0 + 64] = (0.1 + delta * np.cos(ph)).astype(np.float32)
    got = gpu_run(evx_gpu, c0, "periodic", "spectral", n, p)
    amp_num = amp0 = den = 0.0
    mean_got = mean0 = 0.0
    for z0 in range(0, 1024, 64):
        ph = 2 * np.pi * (m[2] * ix / 1024 + m[1] * iy / 1024 + m[0] * iz[z0:z0 + 64] / 1024)
        mode = np.cos(ph)
        amp_num += float(np.sum(got[z0:z0 + 64].astype(np.float64) * mode))
        amp0 += float(np.sum(c0[z0:z0 + 64].astype(np.float64) * mode))
        den += float(np.sum(mode * mode))
        mean_got += float(np.sum(got[z0:z0 + 64], dtype=np.float64))
        mean0 += float(np.sum(c0[z0:z0 + 64], dtype=np.float64))
    K2 = sum(ch.axis_k2(1024, 1.0, "periodic", "spectral")[mi] for mi in m)
    g = ch.growth_factor(K2, mean0 / c0.size, p)
    assert abs((amp_num / den) / ((amp0 / den) * g ** n) - 1.0) <= 2e-3
    assert abs(mean_got - mean0) / c0.size <= 1e-7


def _mirror(block, times):
    out = block
    for _ in range(times):
        for ax in range(3):
            out = np.concatenate([out, np.flip(out, axis=ax)], axis=ax)
    return out


def test_400_zero_flux_mirror_tiled(evx_gpu):
    """400^3 zero flux, stencil: the 25^3 block mirrored four times per axis (400 = 25 * 2^4)
    steps to the mirrored oracle step of the block."""
    p = OParams(dt=0.5)
    small = quench_field((25, 25, 25), 0.0, 0.05, seed=4)
    big = _mirror(small, 4)
    ref = _mirror(ch.ch_run(small, 5, p, "zero_flux", "stencil7"), 4)
    got = gpu_run(evx_gpu, big, "zero_flux", "stencil7", 5, p)
    assert rel_l2(got, ref) <= 1e-5


def test_400_zero_flux_random_one_step(evx_gpu):
    p = OParams(dt=0.5)
    c0 = quench_field((400, 400, 400), 0.0, 0.05, seed=4)
    got = gpu_run(evx_gpu, c0, "zero_flux", "stencil7", 1, p)
    ref = ch.ch_step(c0.astype(np.float64), p, "zero_flux", "stencil7")
    assert rel_l2(got, ref) <= 1e-5


@pytest.mark.parametrize("bc", ["periodic", "zero_flux"])
def test_nonfinite_state_is_reported(evx_gpu, bc):
    """check_finite: a NaN or an Inf in the field makes the step return EVX_ERR_NONFINITE (7);
    a finite field passes the check with results bitwise equal to an unchecked run."""
    shape = (16, 24, 32)
    c0 = quench_field(shape, 0.0, 0.05, seed=7)
    checked = evx_gpu.CHParams(dt=0.5, check_finite=True)
    plain = evx_gpu.CHParams(dt=0.5)
    plan = evx_gpu.Plan(shape, bc, "spectral")
    a = torch.from_numpy(c0).cuda()
    b = torch.from_numpy(c0).cuda()
    plan.step(a, 3, checked)
    plan.step(b, 3, plain)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    for bad in (float("nan"), float("inf"), -float("inf")):
        c = torch.from_numpy(c0).cuda()
        c[5, 7, 11] = bad
        with pytest.raises(evx_gpu.EvxError) as ei:
            plan.step(c, 2, checked)
        assert ei.value.status == 7
        c = torch.from_numpy(c0).cuda()
        c[5, 7, 11] = bad
        plan.step(c, 2, plain)  # unchecked: no status, the field is simply non-finite
        torch.cuda.synchronize()
        assert not bool(torch.isfinite(c).all())
    # a step that makes a finite state overflow is caught at the end of the batch
    big = torch.from_numpy(c0 * 1e13).cuda()
    with pytest.raises(evx_gpu.EvxError) as ei:
        plan.step(big, 4, evx_gpu.CHParams(dt=0.5, A=0.0, check_finite=True))
    assert ei.value.status == 7
