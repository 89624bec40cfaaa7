"""Pins of the FP64 oracle against what the mathematics fixes (no GPU).

Each test ties the oracle to something other than itself:
  * a dense brute-force solve of the step's linear system, with Laplacians assembled from closed
    forms (the periodic spectral second-derivative matrix of the trigonometric interpolant, the
    3-point stencil with wrap or mirrored ghost cells) and no transform at all;
  * the paper's increment form with a real-space stencil right-hand side;
  * the mirror-extension identity (zero-flux step = periodic step on the even extension);
  * conservation of mass, monotone decay of the free energy, the closed-form growth factor and the
    linear growth rate of small modes, first-order convergence in time and second-order (stencil)
    or exact (spectral) behaviour in space on manufactured solutions.
"""
import numpy as np
import pytest

from oracle import ch
from oracle.ch import CHParams
from paper_2507_21748_amd.inputs import mode_field, quench_field

BCS = ["periodic", "zero_flux"]
SCHEMES = ["spectral", "stencil7"]


# --------------------------------------------------------------------------- dense references
def _d2_periodic_spectral(n, dx):
    """Second-derivative matrix of the periodic trigonometric interpolant on n (even) points
    (Trefethen, Spectral Methods in MATLAB, ch. 3): diagonal -pi^2/(3h^2) - 1/6, off-diagonal
    -(-1)^j / (2 sin^2(j h / 2)), h = 2 pi / n, rescaled from [0, 2 pi) to length n dx."""
    assert n % 2 == 0
    h = 2 * np.pi / n
    D = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            d = (i - j) % n
            D[i, j] = (-np.pi ** 2 / (3 * h * h) - 1.0 / 6.0) if d == 0 else \
                -((-1) ** d) / (2 * np.sin(d * h / 2) ** 2)
    return D * (2 * np.pi / (n * dx)) ** 2


def _d2_1d(n, dx, bc, scheme):
    if scheme == "stencil7":
        D = np.zeros((n, n))
        for i in range(n):
            D[i, i] = -2.0
            if bc == "periodic":
                D[i, (i - 1) % n] += 1.0
                D[i, (i + 1) % n] += 1.0
            else:  # cell-centred mirror ghost: u_{-1} = u_0, u_n = u_{n-1}
                D[i, max(i - 1, 0)] += 1.0
                D[i, min(i + 1, n - 1)] += 1.0
        return D / (dx * dx)
    if bc == "periodic":
        return _d2_periodic_spectral(n, dx)
    # zero flux, spectral: restriction of the 2n periodic operator to even extensions about the
    # cell faces, e(j) = c(j), e(2n-1-j) = c(j)
    D2 = _d2_periodic_spectral(2 * n, dx)
    return D2[:n, :n] + D2[:n, ::-1][:, :n]


def _dense_laplacian(shape, dx, bc, scheme):
    nz, ny, nx = shape
    Lz, Ly, Lx = (_d2_1d(n, dx, bc, scheme) for n in (nz, ny, nx))
    Iz, Iy, Ix = np.eye(nz), np.eye(ny), np.eye(nx)
    return (np.kron(Lz, np.kron(Iy, Ix)) + np.kron(Iz, np.kron(Ly, Ix))
            + np.kron(Iz, np.kron(Iy, Lx)))


def _dense_step(c, p, bc, scheme):
    L = _dense_laplacian(c.shape, p.dx, bc, scheme)
    I = np.eye(L.shape[0])
    v = c.reshape(-1)
    lhs = I + p.dt * p.M * p.kappa * (L @ L) - p.A * p.dt * L
    rhs = (I - p.A * p.dt * L) @ v + p.dt * p.M * (L @ (v ** 3 - v))
    return np.linalg.solve(lhs, rhs).reshape(c.shape)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("shape", [(4, 6, 4), (6, 6, 6)])
def test_step_equals_dense_solve(bc, scheme, shape):
    p = CHParams(dx=0.7, dt=0.3, M=0.8, kappa=1.3, A=2.0)
    c = quench_field(shape, 0.1, 0.6, seed=11).astype(np.float64)
    ref = _dense_step(c, p, bc, scheme)
    got = ch.ch_step(c, p, bc, scheme)
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_dense_laplacian_eigenvalues_match_K2(bc, scheme):
    # the symbols the oracle uses are the eigenvalues of the assembled operators
    n, dx = 8, 0.9
    ev = np.sort(-np.linalg.eigvals(_d2_1d(n, dx, bc, scheme)).real)
    assert np.allclose(ev, np.sort(ch.axis_k2(n, dx, bc, scheme)), atol=1e-10)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_increment_form_equals_kspace_form(bc, scheme):
    p = CHParams(dx=1.0, dt=0.5, M=1.0, kappa=1.0, A=2.0)
    c = quench_field((12, 10, 16), 0.2, 0.3, seed=3).astype(np.float64)
    a = ch.ch_step(c, p, bc, scheme)
    b = ch.ch_step_increment(c, p, bc, scheme)
    assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("scheme", SCHEMES)
def test_mirror_extension_identity(scheme):
    """Zero-flux step on n cells = periodic step on the 2n even extension, restricted."""
    p = CHParams(dt=0.5)
    c = quench_field((6, 10, 8), 0.0, 0.5, seed=5).astype(np.float64)
    e = c
    for ax in range(3):
        e = np.concatenate([e, np.flip(e, axis=ax)], axis=ax)
    per = ch.ch_step(e, p, "periodic", scheme)[:6, :10, :8]
    zf = ch.ch_step(c, p, "zero_flux", scheme)
    assert np.max(np.abs(per - zf)) < 1e-13


@pytest.mark.parametrize("bc", BCS)
def test_periodic_tiling_equivariance(bc):
    """A field that repeats (periodic) or mirror-repeats (zero flux) a smaller block steps to the
    repeated step of the block; the GPU tests use this at full size."""
    p = CHParams(dt=0.5)
    small = quench_field((4, 6, 5), 0.1, 0.4, seed=8).astype(np.float64)
    if bc == "periodic":
        big = np.tile(small, (3, 2, 4))
        ref = np.tile(ch.ch_step(small, p, bc, "spectral"), (3, 2, 4))
    else:
        big = small
        for ax in range(3):
            big = np.concatenate([big, np.flip(big, axis=ax)], axis=ax)
        r = ch.ch_step(small, p, bc, "stencil7")
        ref = r
        for ax in range(3):
            ref = np.concatenate([ref, np.flip(ref, axis=ax)], axis=ax)
    got = ch.ch_step(big, p, bc, "spectral" if bc == "periodic" else "stencil7")
    assert np.max(np.abs(got - ref)) < 1e-13


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_mass_conserved(bc, scheme):
    p = CHParams(dt=0.5)
    c = quench_field((16, 12, 10), 0.2, 0.05, seed=2).astype(np.float64)
    m0 = ch.mass(c)
    for _ in range(50):
        c = ch.ch_step(c, p, bc, scheme)
    assert abs(ch.mass(c) - m0) < 1e-11 * c.size


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_energy_monotone_decay(bc, scheme):
    """The linearly stabilised scheme decreases the discrete free energy for A/M >= max|f''|/2
    over the solution's range (Shen & Yang), here A = 2, M = 1, dt = 0.5."""
    p = CHParams(dt=0.5)
    c = quench_field((16, 16, 16), 0.0, 0.05, seed=1).astype(np.float64)
    E = [ch.energy(c, p, bc, scheme)]
    for _ in range(300):
        c = ch.ch_step(c, p, bc, scheme)
        E.append(ch.energy(c, p, bc, scheme))
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E[:-1]))
    assert E[-1] < 0.75 * E[0]         # spinodal decomposition actually happened
    assert np.max(np.abs(c)) < 1.29    # inside the range where the stability bound holds


def _mean_f_cos(cbar, a, c2, c4):
    """Grid mean of f(cbar + a q) for an oscillating factor q with mean 0, zero odd moments,
    mean(q^2) = c2 and mean(q^4) = c4: f = (c^4 - 2 c^2 + 1) / 4 expanded in powers of a q."""
    m2 = cbar ** 2 + a * a * c2
    m4 = cbar ** 4 + 6.0 * cbar ** 2 * a * a * c2 + a ** 4 * c4
    return 0.25 * (m4 - 2.0 * m2 + 1.0)


def _cos_grid(shape, modes, bc):
    """Product over axes of cos(theta_axis): periodic theta = 2 pi m j / n, zero flux
    theta = pi m (j + 1/2) / n (m = 0 gives a constant factor 1)."""
    q = np.ones(shape)
    for ax, (n, m) in enumerate(zip(shape, modes)):
        j = np.arange(n, dtype=np.float64)
        th = 2.0 * np.pi * m * j / n if bc == "periodic" else np.pi * m * (j + 0.5) / n
        sh = [1, 1, 1]
        sh[ax] = n
        q = q * np.cos(th).reshape(sh)
    return q


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("modes", [(0, 0, 3), (2, 0, 1), (1, 3, 2)])
def test_energy_of_cosine_mode_closed_form(bc, scheme, modes):
    """A cosine mode c = cbar + a prod cos(theta) is an eigenvector of every discrete Laplacian
    here (eigenvalue -K2, the sum of the per-axis values), so the gradient term of the free
    energy is (kappa/2) K2 a^2 V mean(q^2) dx^3, and the grid moments of the cosine product are
    those of the continuum (1/2, 3/8 per active axis) as long as 2m and 4m do not alias.  So
    E = dx^3 V [mean f + (kappa/2) K2 a^2 mean(q^2)] in closed form.  A dropped or rescaled
    kappa, a wrong f or a wrong K2 fails it."""
    shape, dx, cbar, a = (12, 10, 16), 0.7, 0.3, 0.4
    p = CHParams(dx=dx, kappa=1.7)
    c = cbar + a * _cos_grid(shape, modes, bc)
    act = sum(1 for m in modes if m)
    c2, c4 = 0.5 ** act, 0.375 ** act
    K2 = sum(ch.axis_k2(n, dx, bc, scheme)[m] for n, m in zip(shape, modes))
    V = float(np.prod(shape))
    ref = dx ** 3 * V * (_mean_f_cos(cbar, a, c2, c4) + 0.5 * p.kappa * K2 * a * a * c2)
    got = ch.energy(c, p, bc, scheme)
    assert abs(got - ref) <= 1e-12 * abs(ref)


@pytest.mark.parametrize("bc", BCS)
def test_stencil_energy_equals_face_loop(bc):
    """7-point scheme: E = dx^3 [sum f(c) + (kappa/2) sum over faces ((c_b - c_a)/dx)^2] with
    every face between two cells counted once; periodic axes wrap, zero-flux axes have no
    boundary faces (mirror ghosts carry no difference).  Plain Python loops over cells and
    faces."""
    shape, dx = (3, 4, 5), 0.9
    p = CHParams(dx=dx, kappa=1.3)
    c = quench_field(shape, 0.1, 0.6, seed=31).astype(np.float64)
    nz, ny, nx = shape
    bulk = 0.0
    grad = 0.0
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                v = c[z, y, x]
                bulk += 0.25 * (v * v - 1.0) ** 2
                for (dz, dy, dxx) in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    z2, y2, x2 = z + dz, y + dy, x + dxx
                    if bc == "periodic":
                        z2, y2, x2 = z2 % nz, y2 % ny, x2 % nx
                    elif z2 >= nz or y2 >= ny or x2 >= nx:
                        continue
                    grad += ((c[z2, y2, x2] - v) / dx) ** 2
    ref = dx ** 3 * (bulk + 0.5 * p.kappa * grad)
    got = ch.energy(c, p, bc, "stencil7")
    assert abs(got - ref) <= 1e-12 * abs(ref)


def test_energy_decay_fails_without_stabilisation():
    """Sanity of the energy pin: with A = 0 and a large step the explicit treatment of f' is
    unstable and the energy rises, so the monotone-decay test can fail."""
    p = CHParams(dt=5.0, A=0.0)
    c = quench_field((16, 16, 16), 0.0, 0.05, seed=1).astype(np.float64)
    E = [ch.energy(c, p, "periodic", "spectral")]
    for _ in range(80):
        c = ch.ch_step(c, p, "periodic", "spectral")
        E.append(ch.energy(c, p, "periodic", "spectral"))
    assert np.any(np.diff(E) > 0) or not np.all(np.isfinite(E))


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("cbar", [0.0, 0.2, 0.6])
@pytest.mark.parametrize("m,n", [((0, 1, 1), 20), ((1, 2, 3), 4)])
def test_linear_growth_factor(bc, scheme, cbar, m, n):
    """A mode of amplitude 1e-7 on a constant background grows by g(K2)^n to O(delta)."""
    p = CHParams(dt=0.5)
    shape = (8, 12, 16)
    delta = 1e-7
    c = mode_field(shape, cbar, 0.0, m, bc).astype(np.float64) + delta * \
        (mode_field(shape, 0.0, 1.0, m, bc).astype(np.float64))
    base = np.full(shape, cbar)
    for _ in range(n):
        c = ch.ch_step(c, p, bc, scheme)
    pert = c - base
    mode = mode_field(shape, 0.0, 1.0, m, bc).astype(np.float64)
    amp = np.sum(pert * mode) / np.sum(mode * mode)
    kz, ky, kx = (ch.axis_k2(s, p.dx, bc, scheme)[mi] for s, mi in zip(shape, m))
    g = ch.growth_factor(kz + ky + kx, cbar, p)
    assert abs(amp / (delta * g ** n) - 1.0) < 1e-5


def test_growth_rate_limit():
    """ln(g)/dt -> lambda(k) = -M k^2 (f''(cbar) + kappa k^2) at first order as dt -> 0."""
    K2, cbar = 0.35, 0.1
    lam = -1.0 * K2 * (ch.fsecond(cbar) + 1.0 * K2)
    errs = []
    for dt in [0.1, 0.05, 0.025, 0.0125]:
        g = ch.growth_factor(K2, cbar, CHParams(dt=dt))
        errs.append(abs(np.log(g) / dt - lam))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 1.0) < 0.1)


def test_growth_factor_literal_numerator_fails():
    """Documented reading: the numerator must carry the stabilisation (1 + A dt K2) C^n.  Without
    it a linearly unstable mode decays, contradicting lambda(k) > 0 (this pin would catch a
    kernel or oracle that drops the term)."""
    p = CHParams(dt=0.5)
    shape, m = (8, 8, 16), (0, 0, 1)
    c = mode_field(shape, 0.0, 1e-7, m, "periodic").astype(np.float64)
    K2 = ch.axis_k2(16, 1.0, "periodic", "spectral")[1]
    assert -K2 * (ch.fsecond(0.0) + K2) > 0            # unstable mode
    c1 = ch.ch_step(c, p, "periodic", "spectral")
    assert np.max(np.abs(c1)) > np.max(np.abs(c))       # and it grows in the oracle


# --------------------------------------------------------------------------- manufactured solutions
def _mms(shape, dx, t, M, kappa, cbar, amp, kvec):
    """c(x,t) = cbar + a(t) cos(k.x), a(t) = amp e^{-t}, and the source s = dc/dt - M lap(mu)
    with mu = c^3 - c - kappa lap c, differentiated analytically."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz) * dx, np.arange(ny) * dx, np.arange(nx) * dx, indexing="ij")
    th = kvec[0] * z + kvec[1] * y + kvec[2] * x
    k2 = sum(k * k for k in kvec)
    a = amp * np.exp(-t)
    c = cbar + a * np.cos(th)
    lap_c = -a * k2 * np.cos(th)
    grad2 = a * a * k2 * np.sin(th) ** 2
    lap_c3 = 3 * c * c * lap_c + 6 * c * grad2
    lap_mu = lap_c3 - lap_c - kappa * (a * k2 * k2 * np.cos(th))
    s = -a * np.cos(th) - M * lap_mu
    return c, s


def _mms_error(shape, dx, dt, T_end, scheme, bc="periodic"):
    p = CHParams(dx=dx, dt=dt, M=1.0, kappa=1.0, A=2.0)
    L = shape[2] * dx
    kvec = (2 * np.pi / (shape[0] * dx), 0.0, 2 * np.pi / L)
    c, _ = _mms(shape, dx, 0.0, p.M, p.kappa, 0.1, 0.3, kvec)
    nsteps = int(round(T_end / dt))
    for n in range(nsteps):
        _, s = _mms(shape, dx, n * dt, p.M, p.kappa, 0.1, 0.3, kvec)
        c = ch.ch_step(c, p, bc, scheme, source=s)
    exact, _ = _mms(shape, dx, nsteps * dt, p.M, p.kappa, 0.1, 0.3, kvec)
    return np.sqrt(np.mean((c - exact) ** 2))


def test_mms_first_order_in_time():
    errs = [_mms_error((12, 4, 12), 1.0, dt, 2.0, "spectral") for dt in (0.1, 0.05, 0.025)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - 1.0) < 0.15), rates


def test_mms_second_order_in_space_stencil():
    """Stencil vs spectral solution at the same small dt; the difference is the stencil's
    spatial error and halves twice per grid halving."""
    diffs = []
    for n in (8, 16, 32):
        dx = 8.0 / n
        shape = (n, 2, n)
        p = CHParams(dx=dx, dt=0.002)
        kvec = (2 * np.pi / 8.0, 0.0, 2 * np.pi / 8.0)
        c0, _ = _mms(shape, dx, 0.0, 1.0, 1.0, 0.1, 0.3, kvec)
        cs, cp = c0.copy(), c0.copy()
        for i in range(50):
            _, s = _mms(shape, dx, i * p.dt, 1.0, 1.0, 0.1, 0.3, kvec)
            cs = ch.ch_step(cs, p, "periodic", "stencil7", source=s)
            cp = ch.ch_step(cp, p, "periodic", "spectral", source=s)
        diffs.append(np.sqrt(np.mean((cs - cp) ** 2)))
    rates = np.log2(np.array(diffs[:-1]) / np.array(diffs[1:]))
    assert np.all(np.abs(rates - 2.0) < 0.2), rates


def test_mms_spectral_space_exact():
    """For a band-limited solution (c^3 resolved) the spectral scheme's error does not depend on
    the grid: only the time error remains."""
    e1 = _mms_error((12, 4, 12), 1.0, 0.05, 1.0, "spectral")
    e2 = _mms_error((24, 4, 24), 0.5, 0.05, 1.0, "spectral")
    assert abs(e1 - e2) < 1e-10 * max(e1, 1e-300) + 1e-14


def test_fp32_sensitivity_small_config():
    """Attainability of the FP32 tolerance at the 32^3 quench: two FP64 runs whose initial
    conditions differ by one float32 ulp differ far less than 1e-3 after 100 steps."""
    p = CHParams(dt=0.1)
    c0 = quench_field((32, 32, 32), 0.0, 0.05, seed=1).astype(np.float64)
    c1 = np.nextafter(c0.astype(np.float32), np.float32(np.inf)).astype(np.float64)
    a = ch.ch_run(c0, 100, p, "periodic", "spectral")
    b = ch.ch_run(c1, 100, p, "periodic", "spectral")
    rel = np.linalg.norm(a - b) / np.linalg.norm(a)
    assert rel < 1e-4, rel
