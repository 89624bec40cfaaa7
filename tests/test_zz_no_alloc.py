"""The allocation-free step (evx_ch_step_noalloc) through the C ABI: on a plan with no workspace,
two calls in a row (the second on a smaller grid, so stale scratch contents from the first are
present) give fields bitwise equal to evx_ch_step's, and a grid beyond the static scratch is
refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

from oracle import ch
from paper_2507_21748_amd.inputs import quench_field

pytestmark = pytest.mark.gpu


def _bare_plan(lib, shape, bc, scheme):
    """A plan created through the C ABI with no workspace set."""
    nz, ny, nx = shape
    h = ctypes.c_void_p()
    st = lib.evx_plan_create(ctypes.byref(h), nx, ny, nz, {"periodic": 0, "zero_flux": 1}[bc],
                             {"spectral": 0, "stencil7": 1}[scheme], ctypes.c_double(1.0))
    assert st == 0, lib.evx_last_error()
    return h


def test_noalloc_step_matches_step(evx_gpu):
    lib = evx_gpu.load()
    params = evx_gpu.CHParams(dt=0.5)
    pc = params.c()
    cases = [((64, 96, 128), "periodic", "spectral", 7),
             ((24, 40, 48), "zero_flux", "stencil7", 4)]   # second call: smaller grid
    for shape, bc, scheme, nsteps in cases:
        print(f"noalloc {shape} {bc} {scheme} x{nsteps}", flush=True)
        c0 = quench_field(shape, 0.1, 0.05, seed=61)
        ref_plan = evx_gpu.Plan(shape, bc, scheme)
        ref = torch.from_numpy(c0).cuda()
        ref_plan.step(ref, nsteps, params)
        h = _bare_plan(lib, shape, bc, scheme)
        try:
            got = torch.from_numpy(c0).cuda()
            st = lib.evx_ch_step_noalloc(h, ctypes.c_void_p(got.data_ptr()), nsteps,
                                         ctypes.byref(pc), None)
            assert st == 0, lib.evx_last_error()
            torch.cuda.synchronize()
            assert torch.equal(got, ref)
            if nsteps == 4:  # and against the oracle, to the stepper's per-step bound
                r = ch.ch_run(c0, nsteps, ch.CHParams(dt=0.5), bc, scheme)
                g64 = got.cpu().numpy().astype(np.float64)
                assert np.linalg.norm(g64 - r) / np.linalg.norm(r) <= 1e-4
        finally:
            lib.evx_plan_destroy(h)


def test_noalloc_rejects_grids_beyond_the_scratch(evx_gpu):
    lib = evx_gpu.load()
    h = _bare_plan(lib, (256, 256, 256), "periodic", "spectral")  # 2 x 71 MB > 64 MiB
    try:
        c = torch.zeros(1, device="cuda")  # never touched: the size check comes first
        pc = evx_gpu.CHParams(dt=0.5).c()
        st = lib.evx_ch_step_noalloc(h, ctypes.c_void_p(c.data_ptr()), 1, ctypes.byref(pc), None)
        assert st == 4, st  # EVX_ERR_NOMEM
        assert b"static scratch" in lib.evx_last_error()
    finally:
        lib.evx_plan_destroy(h)
