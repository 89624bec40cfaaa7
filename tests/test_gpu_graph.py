"""The step loop replayed as captured HIP graphs (evx_plan_set_step_graph) against the same loop
launched kernel by kernel: bitwise equal after every replay, with the library's own eager work
(restore, end) and host synchronisations between the replays, across parameter changes (which
recapture), both boundary families, every z-pass update mode, and the automatic mode."""
import numpy as np
import pytest
import torch

from paper_2507_21748_amd.inputs import quench_field

pytestmark = pytest.mark.gpu

CASES = [
    ((128, 128, 128), "periodic", "spectral"),
    ((64, 48, 80), "zero_flux", "stencil7"),
    ((32, 40, 48), ("periodic", "dirichlet", "zero_flux"), "spectral"),
    ((33, 17, 24), ("zero_flux_vertex", "zero_flux_vertex", "periodic"), "stencil7"),
]


def _trajectory(evx, shape, bc, scheme, mode, chunks, params):
    """Run the chunks (nsteps, params) one after another; after each, end into a fresh field
    (the next advance then restores W from the state) and copy it to the host."""
    plan = evx.Plan(shape, bc, scheme)
    plan.set_step_graph(mode)
    c = torch.from_numpy(quench_field(shape, 0.05, 0.3, seed=91)).cuda()
    plan.begin(c)
    outs = []
    for n, prm in zip(chunks, params):
        plan.advance(n, prm)
        out = torch.empty_like(c)
        plan.end(out)
        torch.cuda.synchronize()
        outs.append(out.cpu().numpy())
    return outs


@pytest.mark.parametrize("shape,bc,scheme", CASES)
def test_graph_replays_are_bitwise_equal(evx_gpu, shape, bc, scheme):
    print(f"step graph {shape} {bc} {scheme}", flush=True)
    p1 = evx_gpu.CHParams(dt=0.5, M=1.0, kappa=1.0, A=2.0)
    p2 = evx_gpu.CHParams(dt=0.25, M=0.9, kappa=1.1, A=1.0)
    # with chunks of 8: 2 replays; 3 eager steps; 3 replays + 1 eager (new parameters:
    # recapture); 1 replay (back to the first parameters: recapture again); 2 replays
    chunks = [16, 3, 25, 8, 16]
    params = [p1, p1, p2, p1, p1]
    eager = _trajectory(evx_gpu, shape, bc, scheme, 0, chunks, params)
    graph = _trajectory(evx_gpu, shape, bc, scheme, 8, chunks, params)
    assert all(np.isfinite(e).all() for e in eager)
    for i, (e, g) in enumerate(zip(eager, graph)):
        assert np.array_equal(e, g), f"chunk {i}: max |diff| {np.max(np.abs(e - g))}"


@pytest.mark.parametrize("integrator,model", [(1, 0), (0, 1), (1, 1)])
def test_graph_every_update_mode(evx_gpu, integrator, model):
    """ETD1, Allen-Cahn and Allen-Cahn ETD1 z-pass updates, automatic mode (a 64^3 grid is
    below the automatic threshold, so the default plan replays graphs)."""
    shape = (64, 64, 64)
    prm = evx_gpu.CHParams(dt=0.5, integrator=integrator, model=model)
    chunks, params = [24, 5, 8], [prm] * 3
    eager = _trajectory(evx_gpu, shape, "periodic", "spectral", 0, chunks, params)
    auto = _trajectory(evx_gpu, shape, "periodic", "spectral", -1, chunks, params)
    for e, a in zip(eager, auto):
        assert np.array_equal(e, a)


def test_graph_with_failure_check_and_workspace_change(evx_gpu):
    shape = (32, 32, 32)
    prm = evx_gpu.CHParams(dt=0.5, check_finite=1)
    c0 = quench_field(shape, 0.0, 0.3, seed=92)
    ref = torch.from_numpy(c0).cuda()
    plan = evx_gpu.Plan(shape, "periodic", "spectral")
    plan.set_step_graph(0)
    plan.step(ref, 32, prm)
    plan = evx_gpu.Plan(shape, "periodic", "spectral")
    plan.set_step_graph(16)
    c = torch.from_numpy(c0).cuda()
    plan.step(c, 32, prm)
    torch.cuda.synchronize()
    assert torch.equal(c, ref)
    # a new workspace discards the captured graph, whose kernels address the old one
    plan.set_workspace(torch.empty(plan.workspace_bytes + 4096, dtype=torch.uint8, device="cuda"))
    c = torch.from_numpy(c0).cuda()
    plan.step(c, 32, prm)
    torch.cuda.synchronize()
    assert torch.equal(c, ref)


def test_step_graph_argument_check(evx_gpu):
    plan = evx_gpu.Plan((16, 16, 16), "periodic", "spectral")
    with pytest.raises(evx_gpu.EvxError) as ei:
        plan.set_step_graph(-2)
    assert ei.value.status == 1
    for k in (-1, 0, 1, 64):
        plan.set_step_graph(k)
