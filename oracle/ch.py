"""FP64 CPU oracle for the stabilised semi-implicit Fourier-spectral Cahn-Hilliard step.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this package: only the test
suite, the smoke check and the CPU-baseline leg of the benchmark call it.  It shares no code with
the HIP library; the only thing both sides share are the seeded inputs.

What it computes (paper, Appendix "Semi-implicit timestepping" and "Phase transformations"):

  * the Cahn-Hilliard problem dc/dt = div(M grad mu), mu = f'(c) - kappa lap(c), with constant M,
    kappa and the double well f(c) = (c^2 - 1)^2 / 4 (so f' = c^3 - c);
  * the semi-implicit Fourier-spectral step in the paper's increment form
        c^{n+1} = c^n + T^{-1}{ dt / (1 - dt S) * T{rhs(c^n)} },
    whose symbol S is the Fourier representation of the implicitly treated linear operator
    (the symbol rule closing the appendix).  Here S = -(M kappa K2^2 + A K2): the fourth-order
    term of the CH instance plus a linear stabilisation A K2 (the constant-coefficient splitting
    Gamma = Gamma_0 + (Gamma - Gamma_0) of the same appendix, applied with Gamma_0 = A);
  * the equivalent one-line k-space form
        C^{n+1} = G * (P * C^n - dt M K2 F^n),  P = 1 + A dt K2,
        G = 1 / (1 + dt M kappa K2^2 + A dt K2),  F^n = T[f'(c^n)],
    which is the plain definition: one linear solve per step of
        (I + dt M kappa L^2 - A dt L) c^{n+1} = (I - A dt L) c^n + dt M L f'(c^n)
    with the discrete Laplacian L that T diagonalises.

T is the 3D DFT (periodic), the separable DCT-II (zero flux on a cell-centred grid, where the
update has homogeneous Neumann data), the separable DST-II (Dirichlet: c and its even
derivatives vanish at the outer cell faces) or the separable DCT-I (zero flux on a vertex-centred
grid, "zero_flux_vertex": n points x_j = j dx including both boundary vertices, mirrored about
them).  The appendix notes that the update inherits
homogeneous boundary data, which is what makes a fast transform applicable.  K2 is the eigenvalue of -L: k^2 for the
spectral Laplacian or (4/dx^2) sin^2(k dx/2) for the 7-point stencil, summed over the three axes.

The exponential stepper (first-order exponential time differencing, ETD1; the paper names
exponential integrators among the time steppers the framework accommodates) keeps the same split
dC/dt = S C + N(C), S = -(M kappa K2^2 + A K2), N = -M K2 F + A K2 C, and steps
        C^{n+1} = exp(dt S) C^n + dt phi1(dt S) N^n,   phi1(z) = (exp(z) - 1) / z,
i.e. in the increment form c^{n+1} = c^n + T^{-1}{ dt phi1(dt S) T{rhs(c^n)} }: the multiplier
dt / (1 - dt S) is replaced by dt phi1(dt S).

The Allen-Cahn model (the paper's first-order-transformation kinetics: linear relaxation of the
same free energy towards its minimum) is dc/dt = -M (f'(c) - kappa lap c), M the kinetic
coefficient.  Its split is S = -(M kappa K2 + A), N = -M F + A C (stabilisation A C rather than
A K2 C), so the semi-implicit step is the linear solve
        ((1 + A dt) I - dt M kappa L) c^{n+1} = (1 + A dt) c^n - dt M f'(c^n)
and the ETD1 step is C' = C + dt phi1(dt S) R with R = -M F - M kappa K2 C.

Both forms are implemented here independently (k-space form with spectral multipliers; increment
form with a real-space 7-point stencil for the stencil scheme) and the tests assert that they agree.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.fft as sfft

__all__ = [
    "CHParams", "axis_k2", "k2_grid", "T", "Tinv", "fprime", "fsecond", "fwell",
    "ch_step", "ch_step_increment", "ch_run", "laplacian", "energy", "mass", "growth_factor",
    "ch_step_etd1", "ch_run_etd1", "growth_factor_etd1", "phi1",
    "ac_step", "ac_step_etd1", "ac_run", "ac_growth_factor", "axis_bcs",
]

WORKERS = 1  # scipy.fft threads; the CPU-baseline leg raises it to the host core count


@dataclass(frozen=True)
class CHParams:
    dx: float = 1.0
    dt: float = 0.1
    M: float = 1.0
    kappa: float = 1.0
    A: float = 2.0


def fwell(c):
    """Double-well bulk free energy density f(c) = (c^2 - 1)^2 / 4."""
    return 0.25 * (c * c - 1.0) ** 2


def fprime(c):
    """f'(c) = c^3 - c."""
    return c * c * c - c


def fsecond(c):
    """f''(c) = 3 c^2 - 1."""
    return 3.0 * c * c - 1.0


def axis_k2(n: int, dx: float, bc: str, scheme: str) -> np.ndarray:
    """Eigenvalues of -d^2/dx^2 along one axis of n cells (float64).

    periodic:  k = 2 pi m' / (n dx), m' = m for m <= n/2 else m - n;
    zero flux: k = pi m / (n dx), m = 0..n-1 (cosine modes of the cell-centred grid);
    dirichlet: k = pi m / (n dx), m = 1..n (sine modes: zero at the outer cell faces);
    zero_flux_vertex: k = pi m / ((n - 1) dx), m = 0..n-1 (cosine modes of the vertex grid, whose
    n points span (n - 1) dx).
    spectral:  k^2;   stencil7: (4 / dx^2) sin^2(k dx / 2), the symbol of the 3-point
    second difference (7 points in 3D).
    """
    m = np.arange(n, dtype=np.float64)
    if bc == "periodic":
        mp = np.where(m <= n // 2, m, m - n)
        k = 2.0 * np.pi * mp / (n * dx)
    elif bc == "zero_flux":
        k = np.pi * m / (n * dx)
    elif bc == "dirichlet":
        k = np.pi * (m + 1.0) / (n * dx)
    elif bc == "zero_flux_vertex":
        k = np.pi * m / ((n - 1) * dx)
    else:
        raise ValueError(f"unknown bc {bc!r}")
    if scheme == "spectral":
        return k * k
    if scheme == "stencil7":
        return (4.0 / (dx * dx)) * np.sin(0.5 * k * dx) ** 2
    raise ValueError(f"unknown scheme {scheme!r}")


def axis_bcs(bc):
    """Per-axis boundary conditions (z, y, x): a name for all three axes, or a 3-tuple of
    'periodic', 'zero_flux' and 'dirichlet' (the transforms are then applied axis by axis; a DCT
    or DST of complex data transforms its real and imaginary parts)."""
    if isinstance(bc, str):
        return (bc, bc, bc)
    bcs = tuple(bc)
    if len(bcs) != 3 or any(b not in ("periodic", "zero_flux", "dirichlet", "zero_flux_vertex")
                            for b in bcs):
        raise ValueError(f"bad per-axis bc {bc!r}")
    return bcs


def k2_grid(shape, dx: float, bc, scheme: str) -> np.ndarray:
    """K2(kz, ky, kx) = sum of the per-axis eigenvalues, shape (nz, ny, nx)."""
    nz, ny, nx = shape
    bz, by, bx = axis_bcs(bc)
    return (axis_k2(nz, dx, bz, scheme)[:, None, None]
            + axis_k2(ny, dx, by, scheme)[None, :, None]
            + axis_k2(nx, dx, bx, scheme)[None, None, :])


def T(c, bc: str):
    """Forward transform, unnormalised: full complex 3D DFT (periodic), 3D DCT-II (zero flux) or
    3D DST-II (Dirichlet)."""
    if not isinstance(bc, str):  # per-axis DFT / DCT-II / DST-II / DCT-I
        out = np.asarray(c)
        for ax, b in enumerate(axis_bcs(bc)):
            if b == "periodic":
                out = sfft.fft(out, axis=ax, workers=WORKERS)
            elif b == "zero_flux_vertex":
                out = sfft.dct(out, type=1, axis=ax, workers=WORKERS)
            else:
                f = sfft.dst if b == "dirichlet" else sfft.dct
                out = f(out, type=2, axis=ax, workers=WORKERS)
        return out
    if bc == "periodic":
        return sfft.fftn(c, workers=WORKERS)
    if bc == "dirichlet":
        return sfft.dstn(c, type=2, workers=WORKERS)
    if bc == "zero_flux_vertex":
        return sfft.dctn(c, type=1, workers=WORKERS)
    return sfft.dctn(c, type=2, workers=WORKERS)


def Tinv(C, bc: str, keep_complex: bool = False):
    """Inverse of T.  The periodic result is real up to round-off; its real part is returned unless
    keep_complex (used by complex-step derivatives, whose data are genuinely complex)."""
    if bc == "periodic":
        out = sfft.ifftn(C, workers=WORKERS)
        return out if keep_complex else out.real
    if not isinstance(bc, str):
        out = np.asarray(C)
        for ax, b in enumerate(axis_bcs(bc)):
            if b == "periodic":
                out = sfft.ifft(out, axis=ax, workers=WORKERS)
            elif b == "zero_flux_vertex":
                out = sfft.idct(out, type=1, axis=ax, workers=WORKERS)
            else:
                f = sfft.idst if b == "dirichlet" else sfft.idct
                out = f(out, type=2, axis=ax, workers=WORKERS)
        return out if (keep_complex or not np.iscomplexobj(out)) else out.real
    if bc == "dirichlet":
        return sfft.idstn(C, type=2, workers=WORKERS)
    if bc == "zero_flux_vertex":
        return sfft.idctn(C, type=1, workers=WORKERS)
    return sfft.idctn(C, type=2, workers=WORKERS)


def ch_step(c, p: CHParams, bc: str, scheme: str, source=None, keep_complex: bool = False):
    """One step in k-space form: C' = G (P C - dt M K2 F) [+ G dt S_src]."""
    K2 = k2_grid(c.shape, p.dx, bc, scheme)
    C = T(c, bc)
    F = T(fprime(c), bc)
    P = 1.0 + p.A * p.dt * K2
    G = 1.0 / (1.0 + p.dt * p.M * p.kappa * K2 * K2 + p.A * p.dt * K2)
    num = P * C - p.dt * p.M * K2 * F
    if source is not None:
        num = num + p.dt * T(source, bc)
    return Tinv(G * num, bc, keep_complex=keep_complex)


def phi1(z):
    """phi1(z) = (exp(z) - 1) / z, with phi1(0) = 1 (expm1 keeps small |z| accurate)."""
    z = np.asarray(z, dtype=np.float64)
    safe = np.where(z == 0.0, 1.0, z)
    return np.where(z == 0.0, 1.0, np.expm1(safe) / safe)


def ch_step_etd1(c, p: CHParams, bc: str, scheme: str, keep_complex: bool = False):
    """One exponential (ETD1) step in increment form:
    C' = C + dt phi1(dt S) R,  S = -(M kappa K2^2 + A K2),  R = T{M L mu} = -M K2 F - M kappa K2^2 C."""
    K2 = k2_grid(c.shape, p.dx, bc, scheme)
    C = T(c, bc)
    F = T(fprime(c), bc)
    S = -(p.M * p.kappa * K2 * K2 + p.A * K2)
    R = -p.M * K2 * F - p.M * p.kappa * K2 * K2 * C
    return Tinv(C + p.dt * phi1(p.dt * S) * R, bc, keep_complex=keep_complex)


def ch_run_etd1(c0, nsteps: int, p: CHParams, bc: str, scheme: str):
    """nsteps ETD1 steps from c0 (float64 copy)."""
    c = np.asarray(c0, dtype=np.float64).copy()
    for _ in range(nsteps):
        c = ch_step_etd1(c, p, bc, scheme)
    return c


def growth_factor_etd1(K2, cbar: float, p: CHParams):
    """Per-step amplification of a small mode on a constant background cbar under ETD1: the
    linearised right-hand side is lam C with lam = -M K2 (f''(cbar) + kappa K2), so
        g = 1 + dt phi1(dt S) lam,  S = -(M kappa K2^2 + A K2)."""
    K2 = np.asarray(K2, dtype=np.float64)
    lam = -p.M * K2 * (fsecond(cbar) + p.kappa * K2)
    S = -(p.M * p.kappa * K2 * K2 + p.A * K2)
    return 1.0 + p.dt * phi1(p.dt * S) * lam


def ac_step(c, p: CHParams, bc: str, scheme: str):
    """One semi-implicit Allen-Cahn step: C' = G (P C - dt M F), P = 1 + A dt,
    G = 1 / (1 + A dt + dt M kappa K2)."""
    K2 = k2_grid(c.shape, p.dx, bc, scheme)
    C = T(c, bc)
    F = T(fprime(c), bc)
    P = 1.0 + p.A * p.dt
    G = 1.0 / (1.0 + p.A * p.dt + p.dt * p.M * p.kappa * K2)
    return Tinv(G * (P * C - p.dt * p.M * F), bc)


def ac_step_etd1(c, p: CHParams, bc: str, scheme: str):
    """One exponential (ETD1) Allen-Cahn step: C' = C + dt phi1(dt S) R,
    S = -(M kappa K2 + A), R = -M F - M kappa K2 C."""
    K2 = k2_grid(c.shape, p.dx, bc, scheme)
    C = T(c, bc)
    F = T(fprime(c), bc)
    S = -(p.M * p.kappa * K2 + p.A)
    R = -p.M * F - p.M * p.kappa * K2 * C
    return Tinv(C + p.dt * phi1(p.dt * S) * R, bc)


def ac_run(c0, nsteps: int, p: CHParams, bc: str, scheme: str, etd1: bool = False):
    """nsteps Allen-Cahn steps from c0 (float64 copy)."""
    step = ac_step_etd1 if etd1 else ac_step
    c = np.asarray(c0, dtype=np.float64).copy()
    for _ in range(nsteps):
        c = step(c, p, bc, scheme)
    return c


def ac_growth_factor(K2, cbar: float, p: CHParams, etd1: bool = False):
    """Per-step amplification of a small mode on a constant background cbar (itself moving only
    at second order when f'(cbar) = 0): the linearised right-hand side is lam C,
    lam = -M (f''(cbar) + kappa K2); semi-implicit g = (1 + A dt - dt M f''(cbar)) /
    (1 + A dt + dt M kappa K2); ETD1 g = 1 + dt phi1(dt S) lam."""
    K2 = np.asarray(K2, dtype=np.float64)
    if etd1:
        lam = -p.M * (fsecond(cbar) + p.kappa * K2)
        return 1.0 + p.dt * phi1(-p.dt * (p.M * p.kappa * K2 + p.A)) * lam
    return (1.0 + p.A * p.dt - p.dt * p.M * fsecond(cbar)) / (
        1.0 + p.A * p.dt + p.dt * p.M * p.kappa * K2)


def laplacian(u, dx: float, bc: str, scheme: str):
    """Discrete Laplacian L u.  stencil7: real-space 3-point second difference per axis with
    periodic wrap or, on the cell-centred grid, a mirrored ghost cell (zero flux: u_{-1} = u_0,
    u_n = u_{n-1}; Dirichlet: u_{-1} = -u_0, u_n = -u_{n-1}, zero at the faces); on the vertex
    grid the mirror is about the boundary vertex (u_{-1} = u_1, u_n = u_{n-2}).  spectral:
    multiplier -K2 through T."""
    if scheme == "spectral":
        return Tinv(-k2_grid(u.shape, dx, bc, scheme) * T(u, bc), bc)
    out = np.zeros_like(u)
    for ax, bca in enumerate(axis_bcs(bc)):
        if bca == "periodic":
            up = np.roll(u, -1, axis=ax)
            dn = np.roll(u, 1, axis=ax)
        else:
            pad = [(0, 0)] * 3
            pad[ax] = (1, 1)
            ue = np.pad(u, pad, mode="reflect" if bca == "zero_flux_vertex" else "edge")
            sl_up = [slice(None)] * 3
            sl_dn = [slice(None)] * 3
            sl_up[ax] = slice(2, None)
            sl_dn[ax] = slice(0, -2)
            if bca == "dirichlet":  # antisymmetric ghosts
                lo = [slice(None)] * 3
                hi = [slice(None)] * 3
                lo[ax] = slice(0, 1)
                hi[ax] = slice(-1, None)
                ue[tuple(lo)] *= -1.0
                ue[tuple(hi)] *= -1.0
            up = ue[tuple(sl_up)]
            dn = ue[tuple(sl_dn)]
        out = out + (up - 2.0 * u + dn)
    return out / (dx * dx)


def ch_step_increment(c, p: CHParams, bc: str, scheme: str, source=None):
    """One step in the paper's increment form with the right-hand side evaluated in real space:
        rhs = M L(f'(c) - kappa L c) [+ s],   c' = c + T^{-1}[ dt / (1 - dt S) T[rhs] ],
        S = -(M kappa K2^2 + A K2)."""
    K2 = k2_grid(c.shape, p.dx, bc, scheme)
    mu = fprime(c) - p.kappa * laplacian(c, p.dx, bc, scheme)
    rhs = p.M * laplacian(mu, p.dx, bc, scheme)
    if source is not None:
        rhs = rhs + source
    S = -(p.M * p.kappa * K2 * K2 + p.A * K2)
    return c + Tinv(p.dt / (1.0 - p.dt * S) * T(rhs, bc), bc)


def ch_run(c0, nsteps: int, p: CHParams, bc: str, scheme: str, every=None):
    """nsteps k-space steps from c0 (float64 copy).  If every is given, also returns the list of
    states at steps 0, every, 2*every, ... (including the last)."""
    c = np.asarray(c0, dtype=np.float64).copy()
    states = [c.copy()] if every else None
    for n in range(nsteps):
        c = ch_step(c, p, bc, scheme)
        if every and ((n + 1) % every == 0 or n + 1 == nsteps):
            states.append(c.copy())
    return (c, states) if every else c


def mass(c, dx: float = 1.0) -> float:
    """Total mass dx^3 * sum(c)."""
    return float(dx ** 3 * np.sum(c, dtype=np.float64))


def energy(c, p: CHParams, bc: str, scheme: str) -> float:
    """Discrete free energy E = dx^3 [ sum f(c) - (kappa/2) sum c L c ] (the Ginzburg-Landau
    functional of the appendix with the step's double well f(c) = (c^2 - 1)^2 / 4; -sum c L c is
    the discrete sum over |grad c|^2, i.e. the face differences for the stencil)."""
    c = np.asarray(c, dtype=np.float64)
    lap = laplacian(c, p.dx, bc, scheme)
    return float(p.dx ** 3 * (np.sum(fwell(c)) - 0.5 * p.kappa * np.sum(c * lap)))


def growth_factor(K2, cbar: float, p: CHParams):
    """Per-step amplification of a small mode with eigenvalue K2 on a constant background cbar:
    linearising f'(cbar + d) = f'(cbar) + f''(cbar) d in the k-space form gives
        g = (1 + dt K2 (A - M f''(cbar))) / (1 + dt M kappa K2^2 + A dt K2)."""
    K2 = np.asarray(K2, dtype=np.float64)
    return ((1.0 + p.dt * K2 * (p.A - p.M * fsecond(cbar)))
            / (1.0 + p.dt * p.M * p.kappa * K2 * K2 + p.A * p.dt * K2))
