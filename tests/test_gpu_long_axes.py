"""Random-field GPU parity at transform lengths 512 and 1024 (the 512^3 and 1024^3 workloads'
kernels) against the FP64 oracle, through the C ABI.

Thin grids put each long axis in every role: y (inverse and forward column passes), z (the fused
z pass with the k-space update) and x (the fused row pass: a 512-point complex FFT for a periodic
row of 1024, a 1024-point Makhoul DCT for a zero-flux row), each for both boundary families.  A
random field populates every bin, so every twiddle entry, exchange index and Makhoul reordering
of these plans takes part (a structured field, e.g. a periodic tiling, leaves most of them
multiplying zeros).  Tolerances: relative L2 over all voxels, 1e-5 after one step and 1e-4 after
ten (the per-step bound and the short-run bound of the stepper's parity tests)."""
import os

import numpy as np
import pytest

from oracle import ch
from oracle.ch import CHParams as OParams
from paper_2507_21748_amd.inputs import quench_field
from tests.test_gpu_ch import gpu_run, rel_l2

pytestmark = pytest.mark.gpu

ch.WORKERS = min(16, os.cpu_count() or 1)

# (nz, ny, nx), boundary, scheme
LONG = [
    ((32, 1024, 64), "periodic", "spectral"),    # col<1024> along y
    ((1024, 32, 64), "periodic", "spectral"),    # col<1024> along z (fused update)
    ((40, 48, 1024), "periodic", "spectral"),    # row<512> (periodic x of 1024)
    ((32, 512, 96), "periodic", "stencil7"),     # col<512> along y
    ((512, 40, 48), "periodic", "spectral"),     # col<512> along z
    ((48, 40, 512), "periodic", "stencil7"),     # row<256> (periodic x of 512)
    ((32, 1024, 64), "zero_flux", "stencil7"),   # zero-flux col<1024> along y
    ((1024, 32, 64), "zero_flux", "spectral"),   # zero-flux col<1024> along z
    ((40, 48, 1024), "zero_flux", "stencil7"),   # zero-flux row<1024> (Makhoul)
    ((40, 512, 48), "zero_flux", "spectral"),    # zero-flux col<512> along y
    ((512, 48, 40), "zero_flux", "stencil7"),    # zero-flux col<512> along z
    ((48, 40, 512), "zero_flux", "spectral"),    # zero-flux row<512>
]


@pytest.mark.parametrize("shape,bc,scheme", LONG)
def test_long_axis_random_field(evx_gpu, shape, bc, scheme):
    print(f"long-axis parity {shape} {bc} {scheme}", flush=True)
    p = OParams(dt=0.5)
    c0 = quench_field(shape, 0.1, 0.3, seed=41)
    one = gpu_run(evx_gpu, c0, bc, scheme, 1, p)
    err1 = rel_l2(one, ch.ch_step(c0.astype(np.float64), p, bc, scheme))
    ten = gpu_run(evx_gpu, c0, bc, scheme, 10, p)
    err10 = rel_l2(ten, ch.ch_run(c0, 10, p, bc, scheme))
    print(f"  1 step {err1:.2e}, 10 steps {err10:.2e}")
    assert err1 <= 1e-5
    assert err10 <= 1e-4
