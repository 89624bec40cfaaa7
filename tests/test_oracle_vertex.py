"""Pins of the oracle's vertex-centred zero-flux grids (n points x_j = j dx including both boundary
vertices, the field mirrored about them; transform DCT-I): the transform against the plain cosine
sums, a dense brute-force solve of the step with Laplacians assembled without any transform (the
3-point stencil with the mirror about the vertex, and the spectral second-derivative matrix of the
2(n - 1)-periodic interpolant restricted to even extensions), the dense Laplacian's eigenvalues,
the extension identity (the vertex step is the periodic step on the even extension of length
2(n - 1)), closed-form cosine-mode growth, and mixes with other boundaries."""
import numpy as np
import pytest

from oracle import ch
from oracle.ch import CHParams
from paper_2507_21748_amd.inputs import mode_field, quench_field
from tests.test_oracle_ch import _d2_periodic_spectral

SCHEMES = ["spectral", "stencil7"]
V = "zero_flux_vertex"


def _dct1_naive(x):
    """X_k = x_0 + (-1)^k x_{n-1} + 2 sum_{j=1}^{n-2} x_j cos(pi j k / (n - 1))."""
    n = len(x)
    X = np.empty(n)
    for k in range(n):
        s = x[0] + (-1) ** k * x[n - 1]
        for j in range(1, n - 1):
            s += 2.0 * x[j] * np.cos(np.pi * j * k / (n - 1))
        X[k] = s
    return X


def test_transform_is_the_dct1_and_round_trips():
    c = quench_field((5, 9, 7), 0.2, 0.4, seed=51).astype(np.float64)
    C = ch.T(c, V)
    ref = c.copy()
    for ax in range(3):
        ref = np.apply_along_axis(_dct1_naive, ax, ref)
    assert np.max(np.abs(C - ref)) < 1e-12
    assert np.max(np.abs(ch.Tinv(C, V) - c)) < 1e-13


def _d2_vertex(n, dx, scheme):
    if scheme == "stencil7":
        D = np.zeros((n, n))
        for i in range(n):
            D[i, i] = -2.0
            D[i, abs(i - 1) if i > 0 else 1] += 1.0           # mirror: u_{-1} = u_1
            D[i, i + 1 if i < n - 1 else n - 2] += 1.0        # u_n = u_{n-2}
        return D / (dx * dx)
    # spectral: the 2(n-1)-periodic operator on even extensions about the vertices,
    # e(j) = c(j), e(2(n-1) - j) = c(j)
    M = 2 * (n - 1)
    D2 = _d2_periodic_spectral(M, dx)
    L = np.zeros((n, n))
    for i in range(n):
        for j in range(M):
            L[i, j if j < n else M - j] += D2[i, j]
    return L


def _dense_vertex_laplacian(shape, dx, scheme, bcs=(V, V, V)):
    from tests.test_oracle_ch import _d2_1d
    mats = [_d2_vertex(n, dx, scheme) if b == V else _d2_1d(n, dx, b, scheme)
            for n, b in zip(shape, bcs)]
    Lz, Ly, Lx = mats
    Iz, Iy, Ix = (np.eye(n) for n in shape)
    return (np.kron(Lz, np.kron(Iy, Ix)) + np.kron(Iz, np.kron(Ly, Ix))
            + np.kron(Iz, np.kron(Iy, Lx)))


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("shape", [(5, 7, 5), (3, 5, 9)])
def test_step_equals_dense_solve(scheme, shape):
    p = CHParams(dx=0.8, dt=0.4, M=0.9, kappa=1.2, A=2.0)
    c = quench_field(shape, 0.1, 0.5, seed=52).astype(np.float64)
    L = _dense_vertex_laplacian(shape, p.dx, scheme)
    I = np.eye(L.shape[0])
    v = c.reshape(-1)
    lhs = I + p.dt * p.M * p.kappa * (L @ L) - p.A * p.dt * L
    rhs = (I - p.A * p.dt * L) @ v + p.dt * p.M * (L @ (v ** 3 - v))
    ref = np.linalg.solve(lhs, rhs).reshape(shape)
    assert np.max(np.abs(ch.ch_step(c, p, V, scheme) - ref)) < 1e-12
    assert np.max(np.abs(ch.ch_step_increment(c, p, V, scheme) - ref)) < 1e-12


@pytest.mark.parametrize("scheme", SCHEMES)
def test_dense_laplacian_eigenvalues_match_K2(scheme):
    shape, dx = (3, 5, 7), 0.9
    L = _dense_vertex_laplacian(shape, dx, scheme)
    ev = np.sort(np.linalg.eigvals(L).real)
    k2 = np.sort(-ch.k2_grid(shape, dx, V, scheme).reshape(-1))
    assert np.max(np.abs(ev - k2)) < 1e-9 * max(1.0, np.max(np.abs(k2)))


@pytest.mark.parametrize("scheme", SCHEMES)
def test_extension_identity(scheme):
    """The vertex step equals the periodic step on the even extension of length 2(n - 1) about
    the boundary vertices, restricted to the n points."""
    p = CHParams(dt=0.5)
    shape = (9, 5, 17)
    c = quench_field(shape, 0.0, 0.5, seed=53).astype(np.float64)
    e = c
    for ax, n in enumerate(shape):
        inner = np.take(e, np.arange(n - 2, 0, -1), axis=ax)
        e = np.concatenate([e, inner], axis=ax)
    assert e.shape == tuple(2 * (n - 1) for n in shape)
    per = ch.ch_step(e, p, "periodic", scheme)[:9, :5, :17]
    assert np.max(np.abs(per - ch.ch_step(c, p, V, scheme))) < 1e-13


@pytest.mark.parametrize("scheme", SCHEMES)
def test_cosine_mode_growth(scheme):
    p = CHParams(dt=0.5)
    shape, m, n, delta = (9, 17, 33), (1, 2, 3), 6, 1e-7
    cbar = 0.1
    mode = mode_field(shape, 0.0, 1.0, m, V).astype(np.float64)
    c = cbar + delta * mode
    for _ in range(n):
        c = ch.ch_step(c, p, V, scheme)
    K2 = sum(ch.axis_k2(s, p.dx, V, scheme)[mi] for s, mi in zip(shape, m))
    amp = np.sum((c - cbar) * mode) / np.sum(mode * mode)
    assert abs(amp / (delta * ch.growth_factor(K2, cbar, p) ** n) - 1) < 1e-5


@pytest.mark.parametrize("bcs", [(V, "zero_flux", "periodic"), ("dirichlet", V, V),
                                 ("periodic", "periodic", V)])
def test_mixed_with_other_boundaries(bcs):
    """Per-axis mixes: the extension identity (even about the vertices along vertex axes, even
    about the faces along zero-flux axes, odd along Dirichlet axes) and a dense solve."""
    p = CHParams(dt=0.5, M=0.9, kappa=1.1, A=2.0)
    shape = (5, 9, 8)
    c = quench_field(shape, 0.0, 0.4, seed=54).astype(np.float64)
    e = c
    for ax, (n, b) in enumerate(zip(shape, bcs)):
        if b == V:
            e = np.concatenate([e, np.take(e, np.arange(n - 2, 0, -1), axis=ax)], axis=ax)
        elif b != "periodic":
            sgn = -1.0 if b == "dirichlet" else 1.0
            e = np.concatenate([e, sgn * np.flip(e, axis=ax)], axis=ax)
    per = ch.ch_step(e, p, "periodic", "spectral")[:5, :9, :8]
    assert np.max(np.abs(per - ch.ch_step(c, p, bcs, "spectral"))) < 1e-12
    if "dirichlet" not in bcs:
        L = _dense_vertex_laplacian(shape, p.dx, "stencil7", bcs)
        I = np.eye(L.shape[0])
        v = c.reshape(-1)
        lhs = I + p.dt * p.M * p.kappa * (L @ L) - p.A * p.dt * L
        rhs = (I - p.A * p.dt * L) @ v + p.dt * p.M * (L @ (v ** 3 - v))
        ref = np.linalg.solve(lhs, rhs).reshape(shape)
        assert np.max(np.abs(ch.ch_step(c, p, bcs, "stencil7") - ref)) < 1e-11
