"""Pins of the oracle's Dirichlet boundary (DST-II on the cell-centred grid): the odd-extension
identity with the periodic step, a dense brute-force solve with Laplacians assembled from
closed-form matrices (antisymmetric ghost cells), the dense Laplacian's eigenvalues against K2, the
closed-form growth of a sine mode, and the exact inverse."""
import numpy as np
import pytest

from oracle import ch
from oracle.ch import CHParams
from paper_2507_21748_amd.inputs import quench_field
from tests.test_oracle_ch import _d2_periodic_spectral

SCHEMES = ["spectral", "stencil7"]


def _d2_dirichlet(n, dx, scheme):
    if scheme == "stencil7":  # ghost u_{-1} = -u_0, u_n = -u_{n-1} (zero at the faces)
        D = np.zeros((n, n))
        for i in range(n):
            D[i, i] = -2.0
            if i > 0:
                D[i, i - 1] += 1.0
            else:
                D[i, i] -= 1.0
            if i + 1 < n:
                D[i, i + 1] += 1.0
            else:
                D[i, i] -= 1.0
        return D / (dx * dx)
    # the 2n periodic operator restricted to odd extensions about the faces, e(2n-1-j) = -c(j)
    D2 = _d2_periodic_spectral(2 * n, dx)
    return D2[:n, :n] - D2[:n, ::-1][:, :n]


def _dense_laplacian(shape, dx, scheme):
    nz, ny, nx = shape
    Lz, Ly, Lx = (_d2_dirichlet(n, dx, scheme) for n in (nz, ny, nx))
    Iz, Iy, Ix = np.eye(nz), np.eye(ny), np.eye(nx)
    return (np.kron(Lz, np.kron(Iy, Ix)) + np.kron(Iz, np.kron(Ly, Ix))
            + np.kron(Iz, np.kron(Iy, Lx)))


def _sine_mode(shape, m):
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    out = np.ones(shape)
    for g, n, mi in zip(grids, shape, m):
        out = out * np.sin(np.pi * mi * (g + 0.5) / n)
    return out


@pytest.mark.parametrize("scheme", SCHEMES)
def test_odd_extension_identity(scheme):
    """Dirichlet step on n cells = periodic step on the 2n odd extension about the cell faces,
    restricted (f' is odd, so the extension is preserved)."""
    p = CHParams(dt=0.5)
    c = quench_field((6, 10, 8), 0.0, 0.5, seed=7).astype(np.float64)
    e = c
    for ax in range(3):
        e = np.concatenate([e, -np.flip(e, axis=ax)], axis=ax)
    per = ch.ch_step(e, p, "periodic", scheme)[:6, :10, :8]
    d = ch.ch_step(c, p, "dirichlet", scheme)
    assert np.max(np.abs(per - d)) < 1e-13


@pytest.mark.parametrize("scheme", SCHEMES)
def test_step_equals_dense_solve(scheme):
    p = CHParams(dx=0.7, dt=0.3, M=0.8, kappa=1.3, A=2.0)
    c = quench_field((4, 6, 4), 0.1, 0.6, seed=8).astype(np.float64)
    L = _dense_laplacian(c.shape, p.dx, scheme)
    I = np.eye(L.shape[0])
    v = c.reshape(-1)
    lhs = I + p.dt * p.M * p.kappa * (L @ L) - p.A * p.dt * L
    rhs = (I - p.A * p.dt * L) @ v + p.dt * p.M * (L @ (v ** 3 - v))
    ref = np.linalg.solve(lhs, rhs).reshape(c.shape)
    got = ch.ch_step(c, p, "dirichlet", scheme)
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("scheme", SCHEMES)
def test_dense_laplacian_eigenvalues_match_K2(scheme):
    shape, dx = (4, 6, 5), 0.9
    ev = np.sort(np.linalg.eigvalsh(-_dense_laplacian(shape, dx, scheme)))
    k2 = np.sort(ch.k2_grid(shape, dx, "dirichlet", scheme).reshape(-1))
    assert np.max(np.abs(ev - k2)) < 1e-9 * k2.max()


@pytest.mark.parametrize("scheme", SCHEMES)
def test_sine_mode_growth(scheme):
    """A sine mode of amplitude 1e-7 on c = 0 grows by g(K2)^n, K2 from its mode numbers."""
    p = CHParams(dt=0.5)
    shape, m, n, delta = (8, 12, 16), (1, 2, 3), 5, 1e-7
    mode = _sine_mode(shape, m)
    c = delta * mode
    for _ in range(n):
        c = ch.ch_step(c, p, "dirichlet", scheme)
    amp = np.sum(c * mode) / np.sum(mode * mode)
    K2 = sum(ch.axis_k2(s_, p.dx, "dirichlet", scheme)[mi - 1] for s_, mi in zip(shape, m))
    assert abs(amp / (delta * ch.growth_factor(K2, 0.0, p) ** n) - 1.0) < 1e-5


def test_transform_round_trip_and_sine_basis():
    c = quench_field((6, 8, 10), 0.2, 0.4, seed=9).astype(np.float64)
    assert np.max(np.abs(ch.Tinv(ch.T(c, "dirichlet"), "dirichlet") - c)) < 1e-13
    C = ch.T(_sine_mode((6, 8, 10), (2, 1, 3)), "dirichlet")
    k = np.unravel_index(np.argmax(np.abs(C)), C.shape)
    assert k == (1, 0, 2)  # bin index m - 1


@pytest.mark.parametrize("scheme", SCHEMES)
def test_increment_form_equals_kspace_form(scheme):
    """The paper's increment form with the real-space Laplacian (antisymmetric ghost cells for the
    stencil) equals the k-space step on Dirichlet grids."""
    p = CHParams(dt=0.3, M=0.9, kappa=1.1, A=1.5)
    c = quench_field((6, 8, 10), 0.1, 0.5, seed=10).astype(np.float64)
    a = ch.ch_step(c, p, "dirichlet", scheme)
    b = ch.ch_step_increment(c, p, "dirichlet", scheme)
    assert np.max(np.abs(a - b)) < 1e-12


def test_stencil_laplacian_against_dense():
    c = quench_field((4, 6, 5), 0.2, 0.5, seed=12).astype(np.float64)
    L = _dense_laplacian(c.shape, 0.8, "stencil7")
    want = (L @ c.reshape(-1)).reshape(c.shape)
    assert np.max(np.abs(ch.laplacian(c, 0.8, "dirichlet", "stencil7") - want)) < 1e-12


MIXES = [("dirichlet", "zero_flux", "zero_flux"), ("zero_flux", "dirichlet", "dirichlet"),
         ("zero_flux", "zero_flux", "dirichlet"), ("dirichlet", "periodic", "periodic"),
         ("zero_flux", "dirichlet", "periodic"), ("periodic", "zero_flux", "periodic"),
         # periodic y or z under a non-periodic x
         ("periodic", "zero_flux", "dirichlet"), ("zero_flux", "periodic", "zero_flux"),
         ("periodic", "periodic", "dirichlet")]


@pytest.mark.parametrize("bcs", MIXES)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_mixed_axes_extension_identity(bcs, scheme):
    """Per-axis boundaries (z, y, x): the step equals the periodic step on the 2n extension that is
    even along zero-flux axes and odd along Dirichlet axes (periodic axes as they are),
    restricted."""
    p = CHParams(dt=0.5)
    c = quench_field((6, 10, 8), 0.0, 0.5, seed=13).astype(np.float64)
    e = c
    for ax, b in enumerate(bcs):
        if b == "periodic":
            continue
        sgn = -1.0 if b == "dirichlet" else 1.0
        e = np.concatenate([e, sgn * np.flip(e, axis=ax)], axis=ax)
    per = ch.ch_step(e, p, "periodic", scheme)[:6, :10, :8]
    got = ch.ch_step(c, p, bcs, scheme)
    assert np.max(np.abs(per - got)) < 1e-13


@pytest.mark.parametrize("bcs", MIXES[:3] + MIXES[6:])
def test_mixed_axes_dense_solve(bcs):
    from tests.test_oracle_ch import _d2_1d
    p = CHParams(dx=0.7, dt=0.3, M=0.8, kappa=1.3, A=2.0)
    c = quench_field((4, 6, 4), 0.1, 0.6, seed=14).astype(np.float64)
    mats = [_d2_dirichlet(n, p.dx, "stencil7") if b == "dirichlet"
            else _d2_1d(n, p.dx, b, "stencil7") for n, b in zip(c.shape, bcs)]
    Lz, Ly, Lx = mats
    Iz, Iy, Ix = (np.eye(n) for n in c.shape)
    L = (np.kron(Lz, np.kron(Iy, Ix)) + np.kron(Iz, np.kron(Ly, Ix))
         + np.kron(Iz, np.kron(Iy, Lx)))
    I = np.eye(L.shape[0])
    v = c.reshape(-1)
    lhs = I + p.dt * p.M * p.kappa * (L @ L) - p.A * p.dt * L
    rhs = (I - p.A * p.dt * L) @ v + p.dt * p.M * (L @ (v ** 3 - v))
    ref = np.linalg.solve(lhs, rhs).reshape(c.shape)
    assert np.max(np.abs(ch.ch_step(c, p, bcs, "stencil7") - ref)) < 1e-12
    assert np.max(np.abs(ch.ch_step_increment(c, p, bcs, "stencil7") - ref)) < 1e-12
