"""Seeded synthetic inputs shared by the HIP path, its tests, the bench and the oracle's tests.

This module holds input generation only (random fields, single Fourier modes, workload
descriptions); it contains none of the time-stepping arithmetic.

Quench recipe: u ~ U[0,1) drawn as float64 from numpy's PCG64 stream with the given seed, in
C order over (nz, ny, nx); c0 = mean + amp * (2u - 1) evaluated in float64 and rounded once to
float32.  Both the GPU path and the FP64 oracle consume these float32 values (the oracle promotes
them to float64), so the two start from bit-identical initial conditions.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = ["quench_field", "mode_field", "surrogate_init", "SURROGATE_LAYERS", "Workload",
           "WORKLOADS"]

_CHUNK = 1 << 24


def quench_field(shape, mean: float, amp: float, seed: int) -> np.ndarray:
    """Seeded quench field of the given (nz, ny, nx) shape as float32, C order.

    Drawn in chunks so that a 1024^3 field never holds the whole float64 draw at once; a PCG64
    stream drawn in chunks equals the same stream drawn in one call.
    """
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape))
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty(n, dtype=np.float32)
    for start in range(0, n, _CHUNK):
        m = min(_CHUNK, n - start)
        u = rng.random(m, dtype=np.float64)
        out[start:start + m] = (mean + amp * (2.0 * u - 1.0)).astype(np.float32)
    return out.reshape(shape)


def mode_field(shape, mean: float, delta: float, m=(1, 0, 0), bc: str = "periodic",
               dx: float = 1.0) -> np.ndarray:
    """Constant background plus one small real Fourier (or cosine) mode, float32.

    m = (mz, my, mx) integer mode numbers.  Periodic: cos(2 pi (mx x/nx + my y/ny + mz z/nz)) at
    grid points x = i dx.  Zero-flux (cell-centred): product of cos(pi m (i + 1/2) / n) over the
    three axes; zero-flux vertex-centred: product of cos(pi m i / (n - 1)).
    """
    nz, ny, nx = (int(s) for s in shape)
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    mz, my, mx = m
    if bc == "periodic":
        ph = 2.0 * np.pi * (mx * ix / nx + my * iy / ny + mz * iz / nz)
        mode = np.cos(ph)
    elif bc == "zero_flux":
        mode = (np.cos(np.pi * mx * (ix + 0.5) / nx) * np.cos(np.pi * my * (iy + 0.5) / ny)
                * np.cos(np.pi * mz * (iz + 0.5) / nz))
    elif bc == "zero_flux_vertex":  # points i dx, i = 0..n-1, both ends on the boundary
        mode = (np.cos(np.pi * mx * ix / (nx - 1)) * np.cos(np.pi * my * iy / (ny - 1))
                * np.cos(np.pi * mz * iz / (nz - 1)))
    else:
        raise ValueError(bc)
    return (mean + delta * mode).astype(np.float32)


# Residual conv net of the learned coarse stepper: (Cin, Cout) per 3x3x3 layer.
SURROGATE_LAYERS = [(1, 32), (32, 32), (32, 32), (32, 1)]


def surrogate_init(seed: int, scale_last: float = 0.1) -> np.ndarray:
    """Seeded initial parameters of the coarse-stepper network as one float32 vector, layer by
    layer W[27, Cout, Cin] then b[Cout]: uniform(-sqrt(6/fan_in), sqrt(6/fan_in)) weights
    (fan_in = 27 Cin), zero biases; the last layer is scaled by scale_last so that the initial
    network is a small perturbation of the identity map."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for li, (ci, co) in enumerate(SURROGATE_LAYERS):
        bound = float(np.sqrt(6.0 / (27 * ci)))
        W = rng.uniform(-bound, bound, size=(27, co, ci))
        if li == len(SURROGATE_LAYERS) - 1:
            W = W * scale_last
        parts += [W.reshape(-1), np.zeros(co)]
    return np.concatenate(parts).astype(np.float32)


@dataclass(frozen=True)
class Workload:
    """One seeded synthetic workload: grid, boundary, wavenumber scheme, physics and IC."""
    name: str
    shape: tuple            # (nz, ny, nx)
    bc: str                 # "periodic" | "zero_flux"
    scheme: str             # "spectral" | "stencil7"
    mean: float
    amp: float
    dt: float
    steps: int
    seed: int
    dx: float = 1.0
    M: float = 1.0
    kappa: float = 1.0
    A: float = 2.0
    extra: dict = field(default_factory=dict)

    @property
    def voxels(self) -> int:
        return int(np.prod(self.shape))

    def initial(self) -> np.ndarray:
        return quench_field(self.shape, self.mean, self.amp, self.seed)


# The five seeded workloads: a 32^3 parity case, the 256^3 off-critical quench (periodic spectral
# and zero-flux stencil variants), the large 1024^3 / 400^3 grids, the 128^3 inverse problem and
# the 512^3 surrogate rollout.
WORKLOADS = {
    "ch32_periodic": Workload("ch32_periodic", (32, 32, 32), "periodic", "spectral",
                              0.0, 0.05, 0.1, 100, 1),
    "ch256_periodic": Workload("ch256_periodic", (256, 256, 256), "periodic", "spectral",
                               0.2, 0.05, 0.5, 1000, 2),
    "ch256_zeroflux": Workload("ch256_zeroflux", (256, 256, 256), "zero_flux", "stencil7",
                               0.2, 0.05, 0.5, 1000, 2),
    "ch1024_periodic": Workload("ch1024_periodic", (1024, 1024, 1024), "periodic", "spectral",
                                0.0, 0.05, 0.5, 200, 3),
    "ch400_zeroflux": Workload("ch400_zeroflux", (400, 400, 400), "zero_flux", "stencil7",
                               0.0, 0.05, 0.5, 200, 4),
    "inverse128": Workload("inverse128", (128, 128, 128), "periodic", "spectral",
                           0.0, 0.05, 0.5, 200, 5,
                           extra={"target_kappa": 1.5, "target_M": 0.8, "checkpoint": 20}),
    "surrogate512": Workload("surrogate512", (512, 512, 512), "periodic", "spectral",
                             0.0, 0.05, 0.5, 1000, 7, extra={"stride": 10}),
}
