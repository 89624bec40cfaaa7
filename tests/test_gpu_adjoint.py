"""GPU adjoint (hand-written, through the C ABI) against the FP64 oracle's adjoint and FP64 finite
differences; checkpointed recomputation against storing every state; diagnostics."""
import os

import numpy as np
import pytest
import torch

from oracle import adjoint, ch
from oracle.ch import CHParams as OParams
from paper_2507_21748_amd.inputs import quench_field

pytestmark = pytest.mark.gpu

ch.WORKERS = min(16, os.cpu_count() or 1)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = [((16, 12, 16), "periodic", "spectral"), ((8, 24, 16), "zero_flux", "stencil7"),
         ((32, 40, 48), "zero_flux", "spectral"), ((24, 32, 20), "periodic", "stencil7"),
         ((16, 12, 16), "dirichlet", "spectral"), ((8, 24, 16), "dirichlet", "stencil7"),
         ((12, 20, 16), ("zero_flux", "dirichlet", "periodic"), "stencil7")]


@pytest.mark.parametrize("shape,bc,scheme", CASES)
def test_one_adjoint_step(evx_gpu, shape, bc, scheme):
    p = OParams(dt=0.5, M=0.8, kappa=1.3, A=2.0)
    c = quench_field(shape, 0.1, 0.4, seed=3)
    lam = quench_field(shape, 0.0, 1.0, seed=4)
    c1 = ch.ch_step(c.astype(np.float64), p, bc, scheme)
    target = c1 - lam.astype(np.float64) / 2          # so that dL/dc^1 = lam
    _, g, dk, dM = adjoint.adjoint_gradients(c, target, 1, p, bc, scheme)
    plan = evx_gpu.Plan(shape, bc, scheme, ops=evx_gpu.OP_STEP | evx_gpu.OP_ADJOINT)
    ct = torch.from_numpy(c).cuda()
    lt = torch.from_numpy(lam).cuda()
    gk = torch.zeros(1, dtype=torch.float64, device="cuda")
    gM = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.adjoint_step(ct, lt, evx_gpu.CHParams(dt=p.dt, M=p.M, kappa=p.kappa, A=p.A), gk, gM)
    torch.cuda.synchronize()
    assert rel(lt.cpu().numpy(), g) <= 1e-5
    assert abs(gk.item() / dk - 1) <= 1e-5
    assert abs(gM.item() / dM - 1) <= 1e-5


@pytest.mark.parametrize("shape,bc,scheme", CASES)
def test_diagnostics(evx_gpu, shape, bc, scheme):
    p = OParams(dt=0.5, kappa=1.3, dx=1.0)
    c = quench_field(shape, 0.2, 0.6, seed=9)
    plan = evx_gpu.Plan(shape, bc, scheme, ops=evx_gpu.OP_STEP | evx_gpu.OP_DIAG)
    out = plan.diagnostics(torch.from_numpy(c).cuda(), evx_gpu.CHParams(kappa=p.kappa)).cpu()
    c64 = c.astype(np.float64)
    assert abs(out[0].item() - ch.mass(c64)) <= 1e-9 * c.size
    assert abs(out[1].item() / ch.energy(c64, p, bc, scheme) - 1) <= 1e-6


def _rollout_grads(evx_gpu, c0, target, shape, bc, scheme, p, nsteps, every):
    from paper_2507_21748_amd.autograd import ch_rollout
    plan = evx_gpu.Plan(shape, bc, scheme, ops=evx_gpu.OP_STEP | evx_gpu.OP_ADJOINT)
    c = torch.from_numpy(c0).cuda().requires_grad_(True)
    kappa = torch.tensor(p.kappa, dtype=torch.float64, requires_grad=True)
    M = torch.tensor(p.M, dtype=torch.float64, requires_grad=True)
    cT = ch_rollout(c, kappa, M, plan, nsteps, p.dt, p.A, every)
    tgt = torch.from_numpy(np.asarray(target, np.float32)).cuda()
    loss = ((cT.double() - tgt.double()) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    return loss.item(), c.grad.cpu().numpy(), kappa.grad.item(), M.grad.item()


@pytest.mark.parametrize("bc,scheme", [("periodic", "spectral"), ("zero_flux", "stencil7"),
                                       ("dirichlet", "spectral")])
def test_rollout_gradients_vs_oracle_and_fd(evx_gpu, bc, scheme):
    """16^3, 40 steps of dt 0.5, checkpoint every 8: gradients w.r.t. c0, kappa, M against the
    oracle's adjoint and FP64 central differences of the oracle's loss (<= 1e-4 relative)."""
    shape, n = (16, 16, 16), 40
    p = OParams(dt=0.5, M=1.0, kappa=1.0, A=2.0)
    c0 = quench_field(shape, 0.0, 0.05, seed=6)
    target = ch.ch_run(c0, n, OParams(dt=0.5, M=0.8, kappa=1.5, A=2.0), bc, scheme)
    L, g, k, M = _rollout_grads(evx_gpu, c0, target, shape, bc, scheme, p, n, 8)
    Lo, go, ko, Mo = adjoint.adjoint_gradients(c0, target, n, p, bc, scheme)
    assert abs(L / Lo - 1) <= 1e-4
    assert abs(k / ko - 1) <= 1e-4
    assert abs(M / Mo - 1) <= 1e-4
    assert rel(g, go) <= 1e-4
    for name, val in (("kappa", k), ("M", M)):
        th = getattr(p, name)
        h = 1e-5
        lp = adjoint.loss_of_params(c0, target, n, adjoint.perturbed(p, **{name: th + h}), bc,
                                    scheme)
        lm = adjoint.loss_of_params(c0, target, n, adjoint.perturbed(p, **{name: th - h}), bc,
                                    scheme)
        fd = (lp - lm) / (2 * h)
        assert abs(val / fd - 1) <= 1e-4, (name, val, fd)
    rng = np.random.default_rng(0)
    v = rng.standard_normal(shape)
    h = 1e-4
    fd = (adjoint.loss_of_params(c0 + h * v, target, n, p, bc, scheme)
          - adjoint.loss_of_params(c0 - h * v, target, n, p, bc, scheme)) / (2 * h)
    assert abs(np.sum(g * v) / fd - 1) <= 1e-4


def test_checkpointing_is_bitwise(evx_gpu):
    shape, n = (16, 24, 32), 30
    p = OParams(dt=0.5)
    c0 = quench_field(shape, 0.1, 0.05, seed=10)
    target = quench_field(shape, 0.1, 0.3, seed=11)
    a = _rollout_grads(evx_gpu, c0, target, shape, "periodic", "spectral", p, n, 1)
    b = _rollout_grads(evx_gpu, c0, target, shape, "periodic", "spectral", p, n, 7)
    c = _rollout_grads(evx_gpu, c0, target, shape, "periodic", "spectral", p, n, 30)
    d = _rollout_grads(evx_gpu, c0, target, shape, "periodic", "spectral", p, n, 0)  # stored
    assert a[0] == b[0] == c[0] == d[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[1], c[1]) and np.array_equal(a[1], d[1])
    assert a[2] == b[2] == c[2] == d[2] and a[3] == b[3] == c[3] == d[3]


@pytest.mark.parametrize("bc,scheme", [("periodic", "spectral"), ("zero_flux", "stencil7")])
def test_adjoint_sweep_equals_single_steps(evx_gpu, bc, scheme):
    """evx_ch_adjoint_sweep over a recorded trajectory is bitwise the loop of single adjoint
    steps (lam and both parameter gradients); nsteps = 0 leaves everything untouched."""
    shape, n = (16, 24, 32), 5
    prm = evx_gpu.CHParams(dt=0.5, M=0.9, kappa=1.1)
    plan = evx_gpu.Plan(shape, bc, scheme, ops=evx_gpu.OP_STEP | evx_gpu.OP_ADJOINT)
    plan.begin(torch.from_numpy(quench_field(shape, 0.1, 0.3, seed=12)).cuda())
    traj = torch.empty((n,) + shape, dtype=torch.float32, device="cuda")
    plan.advance_record(n, prm, traj)
    lam0 = torch.from_numpy(quench_field(shape, 0.0, 1.0, seed=13)).cuda()
    a, b = lam0.clone(), lam0.clone()
    ga = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(2)]
    gb = [torch.zeros(1, dtype=torch.float64, device="cuda") for _ in range(2)]
    for i in range(n - 1, -1, -1):
        plan.adjoint_step(traj[i], a, prm, ga[0], ga[1])
    plan.adjoint_sweep(traj, n, b, prm, gb[0], gb[1])
    plan.adjoint_sweep(traj, 0, b, prm, gb[0], gb[1])
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(ga[0], gb[0]) and torch.equal(ga[1], gb[1])
    assert not torch.equal(a, lam0)
    with pytest.raises(evx_gpu.EvxError) as ei:
        plan.adjoint_sweep(traj, -1, b, prm, gb[0], gb[1])
    assert ei.value.status == 1


def test_inverse_problem_128(evx_gpu):
    """128^3, 200 steps of dt 0.5, checkpoint every 20; target from kappa 1.5, M 0.8; gradients at
    kappa 1, M 1 against the stored oracle gradients (tests/golden/inverse128.npz)."""
    path = os.path.join(GOLDEN, "inverse128.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    gld = np.load(path, allow_pickle=False)
    shape, n = (128, 128, 128), 200
    c0 = quench_field(shape, 0.0, 0.05, seed=5)
    plan = evx_gpu.Plan(shape, "periodic", "spectral")
    t = torch.from_numpy(c0).cuda()
    plan.step(t, n, evx_gpu.CHParams(dt=0.5, M=0.8, kappa=1.5, A=2.0))
    target = t.cpu().numpy()
    assert abs(np.linalg.norm(target) / float(gld["target_norm"]) - 1) <= 1e-5
    L, g, k, M = _rollout_grads(evx_gpu, c0, target, shape, "periodic", "spectral",
                                OParams(dt=0.5), n, 20)
    print(f"128^3 inverse: L {L:.6e}/{float(gld['loss']):.6e} dkappa {k:.6e}/"
          f"{float(gld['dkappa']):.6e} dM {M:.6e}/{float(gld['dM']):.6e}")
    assert abs(L / float(gld["loss"]) - 1) <= 1e-4
    assert abs(k / float(gld["dkappa"]) - 1) <= 1e-4
    assert abs(M / float(gld["dM"]) - 1) <= 1e-4
    gs = g.reshape(-1)[gld["index"]]
    assert np.linalg.norm(gs - gld["grad_c0_sample"]) / np.linalg.norm(gld["grad_c0_sample"]) <= 1e-4
    assert abs(np.linalg.norm(g) / float(gld["grad_c0_norm"]) - 1) <= 1e-4


@pytest.mark.parametrize("bc,scheme", [("periodic", "spectral"), ("zero_flux", "stencil7"),
                                       ("dirichlet", "spectral")])
def test_advance_record_is_bitwise(evx_gpu, bc, scheme):
    """evx_ch_advance_record writes the same c^n as end() after each single step, and leaves the
    same state as plain advancing (bitwise)."""
    shape, n = (16, 24, 32), 6
    prm = evx_gpu.CHParams(dt=0.5)
    c0 = torch.from_numpy(quench_field(shape, 0.1, 0.3, seed=7)).cuda()
    a = evx_gpu.Plan(shape, bc, scheme)
    a.begin(c0)
    ref = []
    for _ in range(n):
        ci = torch.empty_like(c0)
        a.end(ci)
        ref.append(ci)
        a.advance(1, prm)
    b = evx_gpu.Plan(shape, bc, scheme)
    b.begin(c0)
    traj = torch.empty((n,) + shape, dtype=torch.float32, device="cuda")
    b.advance_record(n, prm, traj)
    torch.cuda.synchronize()
    for i in range(n):
        assert torch.equal(traj[i], ref[i]), i
    # the state itself (its whole-tile padding holds whatever the workspace held) through what
    # it determines: the field now and one step later
    for _ in range(2):
        ea, eb = torch.empty_like(c0), torch.empty_like(c0)
        a.end(ea)
        b.end(eb)
        torch.cuda.synchronize()
        assert torch.equal(ea, eb)
        a.advance(1, prm)
        b.advance(1, prm)
