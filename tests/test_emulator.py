"""The HIP pass bodies and pass schedule, compiled for the host and run in the threaded emulator
(tests/emu/emu_main.cpp), against the FP64 oracle (no GPU).

Two builds: AddressSanitizer (every global and LDS buffer is an exactly sized heap allocation,
so any out-of-bounds index in a pass fails here) and ThreadSanitizer (a missing workgroup
barrier around an LDS exchange shows up as a data race).  Builds are cached under _build/emu by
a hash of the sources.
"""
import hashlib
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import ch
from oracle.ch import CHParams
from paper_2507_21748_amd.inputs import quench_field

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_21748_amd", "csrc")
MAIN = os.path.join(ROOT, "tests", "emu", "emu_main.cpp")
OUT = os.path.join(ROOT, "_build", "emu")
SIZES = "X(8) X(12) X(16) X(20) X(24) X(32) X(48) X(64) X(96)"
SAN = {"asan": "-fsanitize=address", "tsan": "-fsanitize=thread"}


def _build(kind: str) -> str:
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hpp"):
            h.update(name.encode())
            h.update(open(os.path.join(CSRC, name), "rb").read())
    h.update(open(MAIN, "rb").read())
    h.update((SIZES + SAN[kind]).encode())
    exe = os.path.join(OUT, f"evx_emu_{kind}_{h.hexdigest()[:16]}")
    if not os.path.exists(exe):
        os.makedirs(OUT, exist_ok=True)
        cmd = [gxx, "-std=c++20", "-O1", "-g", SAN[kind], "-DEVX_HOST_EMULATION",
               "-DEVX_AUX_BLOCKS=3", f"-DEVX_FOR_EACH_N(X)={SIZES}", "-I", CSRC, MAIN,
               "-o", exe + f".tmp{os.getpid()}", "-pthread"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        # a per-process temporary name: parallel test workers may build the same binary
        os.replace(exe + f".tmp{os.getpid()}", exe)
    return exe


@pytest.fixture(scope="module")
def asan():
    return _build("asan")


@pytest.fixture(scope="module")
def tsan():
    return _build("tsan")


def _run(exe, shape, bc, scheme, nsteps, p, c0, remap=1, integrator=0, model=0):
    nz, ny, nx = shape
    with tempfile.TemporaryDirectory() as d:
        c0.astype(np.float32).tofile(os.path.join(d, "in"))
        env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=0")
        code = {"periodic": 0, "zero_flux": 1, "dirichlet": 2, "zero_flux_vertex": 3}
        bcarg = code[bc] if isinstance(bc, str) else \
            1000 + 100 * code[bc[2]] + 10 * code[bc[1]] + code[bc[0]]
        r = subprocess.run([exe, str(nx), str(ny), str(nz), str(bcarg),
                            str(int(scheme == "stencil7")), repr(p.dx), repr(p.dt), repr(p.M),
                            repr(p.kappa), repr(p.A), str(nsteps), str(remap),
                            os.path.join(d, "in"), os.path.join(d, "out"), str(integrator),
                            str(model)],
                           capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
        return np.fromfile(os.path.join(d, "out"), np.float32).reshape(shape)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [
    ((16, 12, 16), "periodic", "spectral", 2),
    ((8, 24, 16), "zero_flux", "stencil7", 2),
    ((20, 16, 24), "periodic", "stencil7", -3),   # resume path: end + restore mid-run
    ((12, 20, 8), "zero_flux", "spectral", -2),
    ((96, 8, 16), "periodic", "spectral", 1),     # three-stage 96-point plan along z
    ((8, 48, 96), "zero_flux", "stencil7", 1),
    ((8, 8, 192), "periodic", "stencil7", 1),     # 96-point packed real rows
    ((64, 12, 16), "periodic", "spectral", 2),    # 64-point plan (4 points per lane) along z
    ((8, 12, 64), "zero_flux", "stencil7", 2),    # ... as the zero-flux row
    ((8, 12, 128), "periodic", "spectral", -2),   # ... as the periodic row (nx/2 = 64), resume
    ((8, 64, 64), "periodic", "spectral", 2),     # plane pass (64 x 64 spectral plane in LDS)
    ((12, 64, 64), "periodic", "stencil7", -3),   # ... stencil K2, resume path
    ((8, 32, 32), "periodic", "spectral", 2),     # ... 32 x 32 planes (68-lane workgroups)
]


@pytest.mark.parametrize("shape,bc,scheme,n", [CASES[0], CASES[1], CASES[2]])
def test_emulated_etd1_matches_oracle(asan, shape, bc, scheme, n):
    """The exponential (ETD1) z-pass update against the oracle's ETD1 steps."""
    p = CHParams(dt=0.5, M=0.9, kappa=1.1, A=2.0)
    c0 = quench_field(shape, 0.1, 0.3, seed=14)
    got = _run(asan, shape, bc, scheme, n, p, c0, integrator=1)
    ref = ch.ch_run_etd1(c0, abs(n), p, bc, scheme)
    assert _rel(got, ref) <= 1e-6


@pytest.mark.parametrize("shape,bc,scheme,n", [CASES[0], CASES[1]])
@pytest.mark.parametrize("etd1", [False, True])
def test_emulated_allen_cahn_matches_oracle(asan, shape, bc, scheme, n, etd1):
    """The Allen-Cahn z-pass updates against the oracle's Allen-Cahn steps."""
    p = CHParams(dt=0.5, M=0.9, kappa=1.1, A=2.0)
    c0 = quench_field(shape, 0.1, 0.3, seed=15)
    got = _run(asan, shape, bc, scheme, n, p, c0, integrator=int(etd1), model=1)
    ref = ch.ac_run(c0, abs(n), p, bc, scheme, etd1=etd1)
    assert _rel(got, ref) <= 1e-6


@pytest.mark.parametrize("bcs", [("dirichlet", "zero_flux", "dirichlet"),
                                 ("zero_flux", "dirichlet", "periodic"),
                                 ("periodic", "zero_flux", "dirichlet"),
                                 ("zero_flux", "periodic", "zero_flux"),
                                 ("periodic", "periodic", "zero_flux")])
def test_emulated_mixed_axes_match_oracle(asan, bcs):
    """Per-axis boundaries (z, y, x) against the oracle, with and without a periodic x, and
    with a periodic y or z under a cosine x (one complex column per x bin)."""
    shape = (12, 20, 16)
    p = CHParams(dt=0.5, M=0.9, kappa=1.1, A=2.0)
    c0 = quench_field(shape, 0.1, 0.3, seed=17)
    got = _run(asan, shape, bcs, "stencil7", 2, p, c0)
    ref = ch.ch_run(c0, 2, p, bcs, "stencil7")
    assert _rel(got, ref) <= 1e-6


VX = "zero_flux_vertex"


@pytest.mark.parametrize("shape,bc,scheme,n", [((9, 13, 17), VX, "spectral", 2),
                                               ((9, 13, 17), VX, "stencil7", -3),
                                               ((9, 12, 16), (VX, "zero_flux", "periodic"),
                                                "stencil7", 2),
                                               ((8, 13, 25), ("dirichlet", VX, VX),
                                                "spectral", 2),
                                               ((12, 16, 25), ("periodic", "periodic", VX),
                                                "spectral", 2),
                                               # vertex z over cosine x (two real x bins per
                                               # column in the z pass)
                                               ((9, 13, 16), (VX, VX, "zero_flux"),
                                                "spectral", 2),
                                               ((13, 12, 16), (VX, "dirichlet", "zero_flux"),
                                                "stencil7", 2)])
def test_emulated_vertex_grids_match_oracle(asan, shape, bc, scheme, n):
    """Vertex-centred zero-flux axes (the periodic transform of the even extension, read
    mirrored and stored cut) against the oracle's DCT-I steps, including the resume path and
    mixes with every other boundary."""
    p = CHParams(dt=0.5, M=0.9, kappa=1.1, A=2.0)
    c0 = quench_field(shape, 0.1, 0.3, seed=18)
    got = _run(asan, shape, bc, scheme, n, p, c0)
    ref = ch.ch_run(c0, abs(n), p, bc, scheme)
    assert _rel(got, ref) <= 1e-6


@pytest.mark.parametrize("shape,scheme,n", [((16, 12, 16), "spectral", 2),
                                             ((20, 16, 24), "stencil7", -3),
                                             ((8, 48, 96), "spectral", 1)])
def test_emulated_dirichlet_matches_oracle(asan, shape, scheme, n):
    """Dirichlet grids (zero-flux kernels on the sign-alternated field, reversed K2) against the
    oracle's DST-II steps, including the resume path."""
    p = CHParams(dt=0.5, M=0.9, kappa=1.1, A=2.0)
    c0 = quench_field(shape, 0.1, 0.3, seed=16)
    got = _run(asan, shape, "dirichlet", scheme, n, p, c0)
    ref = ch.ch_run(c0, abs(n), p, "dirichlet", scheme)
    assert _rel(got, ref) <= 1e-6


@pytest.mark.parametrize("shape,bc,scheme,n", CASES)
def test_emulated_passes_match_oracle(asan, shape, bc, scheme, n):
    p = CHParams(dt=0.5, M=0.9, kappa=1.1, A=2.0)
    c0 = quench_field(shape, 0.1, 0.3, seed=13)
    got = _run(asan, shape, bc, scheme, n, p, c0)
    ref = ch.ch_run(c0, abs(n), p, bc, scheme)
    assert _rel(got, ref) <= 1e-6


def test_emulated_remap_is_a_permutation(asan):
    p = CHParams(dt=0.5)
    c0 = quench_field((24, 16, 48), 0.0, 0.2, seed=14)
    a = _run(asan, (24, 16, 48), "periodic", "spectral", 2, p, c0, remap=1)
    b = _run(asan, (24, 16, 48), "periodic", "spectral", 2, p, c0, remap=0)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("shape,bc,scheme", [((24, 12, 48), "periodic", "spectral"),
                                             ((8, 24, 16), "zero_flux", "stencil7")])
def test_emulated_passes_race_free(tsan, shape, bc, scheme):
    p = CHParams(dt=0.5)
    c0 = quench_field(shape, 0.1, 0.3, seed=15)
    got = _run(tsan, shape, bc, scheme, 1, p, c0)
    assert _rel(got, ch.ch_step(c0.astype(np.float64), p, bc, scheme)) <= 1e-6


def test_planted_missing_barrier_is_caught(tmp_path):
    """Meta-check of the race detector: the same build with the barrier after the LDS writes of
    each FFT stage removed (a copy of the sources, on the CPU only) must be reported."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "csrc"
    shutil.copytree(CSRC, src)
    fft = (src / "evx_fft.hpp").read_text()
    planted = fft.replace("    if constexpr (s < S - 1) evx_sync();\n", "")
    assert planted != fft
    (src / "evx_fft.hpp").write_text(planted)
    exe = tmp_path / "emu_planted"
    r = subprocess.run([gxx, "-std=c++20", "-O1", "-g", "-fsanitize=thread",
                        "-DEVX_HOST_EMULATION", "-DEVX_FOR_EACH_N(X)=X(12) X(24)",
                        "-I", str(src), MAIN, "-o", str(exe), "-pthread"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    c0 = quench_field((24, 24, 48), 0.1, 0.3, seed=15)   # two-stage 24-point transforms
    with tempfile.TemporaryDirectory() as d:
        c0.tofile(os.path.join(d, "in"))
        rr = subprocess.run([str(exe), "48", "24", "24", "0", "0", "1", "0.5", "1", "1", "2", "1",
                             "1", os.path.join(d, "in"), os.path.join(d, "out")],
                            capture_output=True, text=True, timeout=600,
                            env=dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert rr.returncode != 0 or "ThreadSanitizer" in rr.stderr


@pytest.mark.parametrize("shape,bc,scheme", [((16, 12, 16), "periodic", "spectral"),
                                             ((8, 24, 16), "zero_flux", "stencil7"),
                                             ((12, 16, 20), "zero_flux", "spectral"),
                                             ((12, 20, 16), ("zero_flux", "dirichlet",
                                                             "periodic"), "stencil7"),
                                             ((12, 20, 16), ("dirichlet", "zero_flux",
                                                             "dirichlet"), "spectral"),
                                             ((12, 20, 16), ("periodic", "dirichlet",
                                                             "zero_flux"), "stencil7")])
def test_emulated_adjoint_step_and_diagnostics(asan, shape, bc, scheme):
    """One adjoint step (lam, dL/dkappa, dL/dM) and the mass/energy diagnostics of the emulated
    kernels against the oracle's adjoint and energy."""
    from oracle import adjoint
    p = CHParams(dt=0.5, M=0.8, kappa=1.3, A=2.0)
    c = quench_field(shape, 0.1, 0.4, seed=3)
    lam = quench_field(shape, 0.0, 1.0, seed=4)
    c1 = ch.ch_step(c.astype(np.float64), p, bc, scheme)
    _, g, dk, dM = adjoint.adjoint_gradients(c, c1 - lam.astype(np.float64) / 2, 1, p, bc, scheme)
    nz, ny, nx = shape
    code = {"periodic": 0, "zero_flux": 1, "dirichlet": 2}
    bcarg = code[bc] if isinstance(bc, str) else \
        1000 + 100 * code[bc[2]] + 10 * code[bc[1]] + code[bc[0]]
    geo = [str(nx), str(ny), str(nz), str(bcarg), str(int(scheme == "stencil7")), "1"]
    with tempfile.TemporaryDirectory() as d:
        c.tofile(os.path.join(d, "c"))
        lam.tofile(os.path.join(d, "l"))
        r = subprocess.run([asan, "adj", *geo, repr(p.dt), repr(p.M), repr(p.kappa), repr(p.A),
                            os.path.join(d, "c"), os.path.join(d, "l"), os.path.join(d, "lo"),
                            os.path.join(d, "g")], capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        lo = np.fromfile(os.path.join(d, "lo"), np.float32).reshape(shape)
        gr = np.fromfile(os.path.join(d, "g"), np.float64)
        r = subprocess.run([asan, "diag", *geo, repr(p.kappa), os.path.join(d, "c"),
                            os.path.join(d, "o")], capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        o = np.fromfile(os.path.join(d, "o"), np.float64)
    assert _rel(lo, g) <= 1e-6
    assert abs(gr[0] / dk - 1) <= 2e-6 and abs(gr[1] / dM - 1) <= 2e-6
    assert abs(o[0] - ch.mass(c.astype(np.float64))) <= 1e-9 * c.size
    assert abs(o[1] / ch.energy(c.astype(np.float64), p, bc, scheme) - 1) <= 1e-6


@pytest.mark.parametrize("shape,bc,scheme", [((16, 12, 16), "periodic", "stencil7"),
                                             ((8, 24, 16), "zero_flux", "spectral"),
                                             ((12, 20, 16), ("dirichlet", "zero_flux",
                                                             "periodic"), "spectral")])
def test_emulated_reaction_diffusion_matches_oracle(asan, shape, bc, scheme):
    """The reaction-diffusion schedule (the fused x pass with the cubic reaction, the z pass's
    update) against the oracle; the Dirichlet mix runs an odd reaction."""
    from oracle import reaction_diffusion as rd
    odd = not isinstance(bc, str)
    p = rd.RDParams(dt=0.4, D=0.8, A=0.5, a0=0.0 if odd else 0.05, a1=0.7,
                    a2=0.0 if odd else -0.6, a3=-0.9)
    c0 = quench_field(shape, 0.3, 0.3, seed=35)
    nz, ny, nx = shape
    code = {"periodic": 0, "zero_flux": 1, "dirichlet": 2}
    bcarg = code[bc] if isinstance(bc, str) else \
        1000 + 100 * code[bc[2]] + 10 * code[bc[1]] + code[bc[0]]
    with tempfile.TemporaryDirectory() as d:
        c0.tofile(os.path.join(d, "c"))
        r = subprocess.run([asan, "rd", str(nx), str(ny), str(nz), str(bcarg),
                            str(int(scheme == "stencil7")), "1.0", repr(p.dt), repr(p.D),
                            repr(p.A), repr(p.a0), repr(p.a1), repr(p.a2), repr(p.a3), "3",
                            os.path.join(d, "c"), os.path.join(d, "o")],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        out = np.fromfile(os.path.join(d, "o"), np.float32).reshape(shape)
    ref = rd.rd_run(c0, 3, p, bc, scheme)
    assert _rel(out, ref) <= 1e-6


@pytest.mark.parametrize("shape,bc,scheme", [((16, 12, 16), "periodic", "spectral"),
                                             ((8, 24, 16), "zero_flux", "stencil7"),
                                             ((12, 20, 16), ("dirichlet", "zero_flux",
                                                             "periodic"), "spectral")])
def test_emulated_gray_scott_matches_oracle(asan, shape, bc, scheme):
    """The Gray-Scott schedule (reaction kernel, batched transforms of four fields, spectral
    update, batched inverse of two) against the oracle's two-species steps."""
    from oracle import gray_scott as gs
    p = gs.GSParams(dt=0.8)
    u0 = quench_field(shape, 0.7, 0.3, seed=31)
    v0 = quench_field(shape, 0.2, 0.2, seed=32)
    nz, ny, nx = shape
    code = {"periodic": 0, "zero_flux": 1, "dirichlet": 2}
    bcarg = code[bc] if isinstance(bc, str) else \
        1000 + 100 * code[bc[2]] + 10 * code[bc[1]] + code[bc[0]]
    with tempfile.TemporaryDirectory() as d:
        u0.tofile(os.path.join(d, "u"))
        v0.tofile(os.path.join(d, "v"))
        r = subprocess.run([asan, "gs", str(nx), str(ny), str(nz), str(bcarg),
                            str(int(scheme == "stencil7")), "1.0", repr(p.dt), repr(p.Du),
                            repr(p.Dv), repr(p.F), repr(p.k), "3", os.path.join(d, "u"),
                            os.path.join(d, "v"), os.path.join(d, "uo"), os.path.join(d, "vo")],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        uo = np.fromfile(os.path.join(d, "uo"), np.float32).reshape(shape)
        vo = np.fromfile(os.path.join(d, "vo"), np.float32).reshape(shape)
    ur, vr = gs.gs_run(u0, v0, 3, p, bc, scheme)
    assert _rel(uo, ur) <= 1e-6 and _rel(vo, vr) <= 1e-6


def _vm_emulated(exe, shape, bc, scheme):
    """Three variable-mobility steps in the emulator and in the oracle: (emulated, oracle, start)."""
    from oracle import ch_varmob as vm
    p = vm.VMParams(dt=0.5, D0=1.2, gamma0=0.9, eps=1.8, M0=0.3)
    phi0 = quench_field(shape, 0.5, 0.2, seed=41)
    nz, ny, nx = shape
    code = {"periodic": 0, "zero_flux": 1}
    bcarg = code[bc] if isinstance(bc, str) else \
        1000 + 100 * code[bc[2]] + 10 * code[bc[1]] + code[bc[0]]
    with tempfile.TemporaryDirectory() as d:
        phi0.tofile(os.path.join(d, "phi"))
        r = subprocess.run([exe, "vm", str(nx), str(ny), str(nz), str(bcarg),
                            str(int(scheme == "stencil7")), "1.0", repr(p.dt), repr(p.D0),
                            repr(p.gamma0), repr(p.eps), repr(p.M0), "3",
                            os.path.join(d, "phi"), os.path.join(d, "out")],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        out = np.fromfile(os.path.join(d, "out"), np.float32).reshape(shape)
    return out, vm.vm_run(phi0, 3, p, bc, scheme), phi0


@pytest.mark.parametrize("shape,bc,scheme", [((16, 12, 16), "periodic", "spectral"),
                                             ((20, 48, 64), "periodic", "stencil7"),
                                             ((8, 24, 16), "zero_flux", "stencil7"),
                                             ((12, 20, 16), ("zero_flux", "periodic",
                                                             "periodic"), "stencil7")])
def test_emulated_variable_mobility_matches_oracle(asan, shape, bc, scheme):
    """The variable-mobility schedule against the oracle's increment steps: the fused z-marching
    stencil pass (one grid smaller than a block's column, one with several columns and a short
    last z range; zero-flux axes with their clamped ghosts), then the forward transform, spectral
    multiplier, inverse transform and add."""
    out, ref, phi0 = _vm_emulated(asan, shape, bc, scheme)
    assert np.max(np.abs(ref - phi0)) > 1e-3  # the steps moved the field
    assert _rel(out, ref) <= 1e-6


def test_emulated_fused_stencil_race_free(tsan):
    """The fused stencil pass's LDS rings under the thread sanitizer (every plane's three
    barriers)."""
    out, ref, _ = _vm_emulated(tsan, (20, 48, 64), "periodic", "stencil7")
    assert _rel(out, ref) <= 1e-6
