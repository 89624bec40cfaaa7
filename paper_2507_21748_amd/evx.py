"""Python binding of libevx (ctypes).  Argument marshalling only: every step of the path runs in
the library's HIP kernels; PyTorch supplies device memory and the current stream.

There is no CPU fallback: if the built library is missing, load() raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

__all__ = ["EvxError", "load", "lib_path", "CHParams", "Plan", "BC", "SCHEME", "SEMI_IMPLICIT",
           "ETD1", "CAHN_HILLIARD", "ALLEN_CAHN", "GSParams", "OP_GRAY_SCOTT",
           "VMParams", "OP_VAR_MOBILITY"]

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB = None

BC = {"periodic": 0, "zero_flux": 1, "dirichlet": 2, "zero_flux_vertex": 3}
SCHEME = {"spectral": 0, "stencil7": 1}

OP_STEP, OP_DIAG, OP_ADJOINT, OP_GRAY_SCOTT, OP_VAR_MOBILITY = 1, 2, 4, 8, 16


class EvxError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("M", ctypes.c_double), ("kappa", ctypes.c_double),
                ("A", ctypes.c_double), ("integrator", ctypes.c_int), ("model", ctypes.c_int),
                ("check_finite", ctypes.c_int)]


SEMI_IMPLICIT, ETD1 = 0, 1  # evx_integrator
CAHN_HILLIARD, ALLEN_CAHN = 0, 1  # evx_model


@dataclass(frozen=True)
class CHParams:
    dt: float = 0.1
    M: float = 1.0
    kappa: float = 1.0
    A: float = 2.0
    integrator: int = SEMI_IMPLICIT
    model: int = CAHN_HILLIARD
    check_finite: bool = False  # advance synchronises and raises on a NaN / Inf state

    def c(self) -> _Params:
        return _Params(self.dt, self.M, self.kappa, self.A, self.integrator, self.model,
                       int(bool(self.check_finite)))


class _GSParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("Du", ctypes.c_double), ("Dv", ctypes.c_double),
                ("F", ctypes.c_double), ("k", ctypes.c_double)]


@dataclass(frozen=True)
class GSParams:
    """Gray-Scott (feed F, kill k): du/dt = Du lap u - u v^2 + F (1 - u),
    dv/dt = Dv lap v + u v^2 - k v."""
    dt: float = 1.0
    Du: float = 0.2
    Dv: float = 0.1
    F: float = 0.04
    k: float = 0.10

    def c(self) -> _GSParams:
        return _GSParams(self.dt, self.Du, self.Dv, self.F, self.k)


class _RDParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("D", ctypes.c_double), ("A", ctypes.c_double),
                ("a0", ctypes.c_double), ("a1", ctypes.c_double), ("a2", ctypes.c_double),
                ("a3", ctypes.c_double)]


@dataclass(frozen=True)
class RDParams:
    """Reaction-diffusion: dc/dt = D lap c + a0 + a1 c + a2 c^2 + a3 c^3 (default: logistic
    growth c (1 - c)), stabilisation A."""
    dt: float = 0.5
    D: float = 1.0
    A: float = 0.0
    a0: float = 0.0
    a1: float = 1.0
    a2: float = -1.0
    a3: float = 0.0

    def c(self) -> _RDParams:
        return _RDParams(self.dt, self.D, self.A, self.a0, self.a1, self.a2, self.a3)


class _VMParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("D0", ctypes.c_double), ("gamma0", ctypes.c_double),
                ("eps", ctypes.c_double), ("M0", ctypes.c_double)]


@dataclass(frozen=True)
class VMParams:
    """Variable-mobility Cahn-Hilliard: dphi/dt = div(M grad mu), M = D0 phi (1 - phi),
    mu = gamma0 (18 / eps) phi (1 - phi) (1 - 2 phi) - 2 gamma0 eps lap phi; M0 is the constant
    mobility of the implicit part."""
    dt: float = 0.05
    D0: float = 1.0
    gamma0: float = 1.0
    eps: float = 2.0
    M0: float = 0.25

    def c(self) -> _VMParams:
        return _VMParams(self.dt, self.D0, self.gamma0, self.eps, self.M0)


def lib_path() -> str:
    return os.path.join(_PKG, "libevx.so")


_PROTOS = {
    "evx_plan_create_axes": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                             ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.c_double],
    "evx_plan_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                        ctypes.c_int, ctypes.c_int, ctypes.c_double],
    "evx_plan_destroy": [ctypes.c_void_p],
    "evx_plan_workspace_bytes": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
    "evx_plan_set_workspace": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t],
    "evx_plan_state": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                       ctypes.POINTER(ctypes.c_size_t)],
    "evx_ch_begin": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "evx_ch_advance": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(_Params), ctypes.c_void_p],
    "evx_gs_step": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                    ctypes.POINTER(_GSParams), ctypes.c_void_p],
    "evx_vm_step": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(_VMParams),
                    ctypes.c_void_p],
    "evx_rd_step": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(_RDParams),
                    ctypes.c_void_p],
    "evx_ch_advance_record": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(_Params),
                              ctypes.c_void_p, ctypes.c_void_p],
    "evx_ch_end": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "evx_ch_restore": [ctypes.c_void_p, ctypes.c_void_p],
    "evx_ch_step": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(_Params),
                    ctypes.c_void_p],
    "evx_ch_step_noalloc": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                            ctypes.POINTER(_Params), ctypes.c_void_p],
    "evx_plan_enable_pass_timing": [ctypes.c_void_p, ctypes.c_int],
    "evx_plan_read_pass_times": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                 ctypes.POINTER(ctypes.c_longlong)],
    "evx_plan_set_xcd_remap": [ctypes.c_void_p, ctypes.c_int],
    "evx_plan_set_step_graph": [ctypes.c_void_p, ctypes.c_int],
    "evx_plan_set_plane_pass": [ctypes.c_void_p, ctypes.c_int],
    "evx_ch_adjoint_step": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_void_p],
    "evx_ch_adjoint_sweep": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                             ctypes.POINTER(_Params), ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_void_p],
    "evx_ch_diagnostics": [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Params),
                           ctypes.c_void_p, ctypes.c_void_p],
    "evx_ch_distance": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                        ctypes.c_void_p],
}


def load():
    """Load libevx.so (built in-tree by build()); raises if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(there is no fallback path)")
    lib = ctypes.CDLL(path)
    for name, args in _PROTOS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.evx_status_string.argtypes = [ctypes.c_int]
    lib.evx_status_string.restype = ctypes.c_char_p
    lib.evx_last_error.argtypes = []
    lib.evx_last_error.restype = ctypes.c_char_p
    _LIB = lib
    return lib


def _check(status: int, where: str):
    if status != 0:
        msg = _LIB.evx_last_error().decode(errors="replace")
        raise EvxError(status, where, msg)


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t: torch.Tensor, dtype=torch.float32, numel=None):
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if t.dtype != dtype:
        raise ValueError(f"tensor must be {dtype}")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"tensor has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A grid (nz, ny, nx) with boundary condition and wavenumber scheme, plus its workspace.
    bc is a name for all axes or a (bc_z, bc_y, bc_x) tuple mixing "zero_flux" and "dirichlet"."""

    def __init__(self, shape, bc: str = "periodic", scheme: str = "spectral", dx: float = 1.0,
                 ops: int = OP_STEP, device=None):
        lib = load()
        self.shape = tuple(int(s) for s in shape)
        self.bc, self.scheme, self.dx = bc, scheme, float(dx)
        nz, ny, nx = self.shape
        self.voxels = nx * ny * nz
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.device = dev
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            if isinstance(bc, str):
                _check(lib.evx_plan_create(ctypes.byref(h), nx, ny, nz, BC[bc], SCHEME[scheme],
                                           self.dx), "evx_plan_create")
            else:
                bz, by, bx = (BC[b] for b in bc)
                _check(lib.evx_plan_create_axes(ctypes.byref(h), nx, ny, nz, bx, by, bz,
                                                SCHEME[scheme], self.dx), "evx_plan_create_axes")
        self._h = h
        nb = ctypes.c_size_t()
        _check(lib.evx_plan_workspace_bytes(h, ops, ctypes.byref(nb)), "evx_plan_workspace_bytes")
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr()
        self._ws_off = (-base) % 256
        _check(lib.evx_plan_set_workspace(h, ctypes.c_void_p(base + self._ws_off), nb.value),
               "evx_plan_set_workspace")
        self.workspace_bytes = nb.value

    def set_workspace(self, buf: torch.Tensor):
        """Use the uint8 device tensor buf (at least workspace_bytes + 255 bytes) as the plan's
        workspace; the plan keeps a reference.  Begin or restore a state afterwards."""
        if buf.dtype != torch.uint8 or buf.device != self.device or not buf.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 tensor on the plan's device")
        off = (-buf.data_ptr()) % 256
        if buf.numel() < off + self.workspace_bytes:
            raise ValueError(f"workspace needs {self.workspace_bytes} bytes after alignment")
        _check(_LIB.evx_plan_set_workspace(self._h, ctypes.c_void_p(buf.data_ptr() + off),
                                           self.workspace_bytes), "evx_plan_set_workspace")
        self.workspace, self._ws_off = buf, off

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _LIB is not None:
            _LIB.evx_plan_destroy(h)
            self._h = None

    # ------------------------------------------------------------------ stepping
    def step(self, c: torch.Tensor, nsteps: int, params: CHParams, stream=None):
        """In place: c <- nsteps steps of c."""
        p = params.c()
        _check(_LIB.evx_ch_step(self._h, _dev_ptr(c, numel=self.voxels), int(nsteps),
                                ctypes.byref(p), _stream_handle(stream)), "evx_ch_step")
        return c

    def begin(self, c: torch.Tensor, stream=None):
        _check(_LIB.evx_ch_begin(self._h, _dev_ptr(c, numel=self.voxels), _stream_handle(stream)),
               "evx_ch_begin")

    def advance(self, nsteps: int, params: CHParams, stream=None):
        p = params.c()
        _check(_LIB.evx_ch_advance(self._h, int(nsteps), ctypes.byref(p), _stream_handle(stream)),
               "evx_ch_advance")

    def gs_step(self, u: torch.Tensor, v: torch.Tensor, nsteps: int, params: GSParams,
                stream=None):
        """Advance the Gray-Scott fields u, v (float32 device tensors of the grid) nsteps in place;
        the plan needs ops including OP_GRAY_SCOTT."""
        p = params.c()
        _check(_LIB.evx_gs_step(self._h, _dev_ptr(u, numel=self.voxels),
                                _dev_ptr(v, numel=self.voxels), int(nsteps), ctypes.byref(p),
                                _stream_handle(stream)), "evx_gs_step")
        return u, v

    def vm_step(self, phi: torch.Tensor, nsteps: int, params: VMParams, stream=None):
        """Advance the variable-mobility Cahn-Hilliard field phi (float32 device tensor of the
        grid) nsteps in place; the plan needs ops including OP_VAR_MOBILITY."""
        p = params.c()
        _check(_LIB.evx_vm_step(self._h, _dev_ptr(phi, numel=self.voxels), int(nsteps),
                                ctypes.byref(p), _stream_handle(stream)), "evx_vm_step")
        return phi

    def rd_step(self, c: torch.Tensor, nsteps: int, params: RDParams, stream=None):
        """Advance the reaction-diffusion field c (float32 device tensor of the grid) nsteps in
        place on the plan's state and work buffers."""
        p = params.c()
        _check(_LIB.evx_rd_step(self._h, _dev_ptr(c, numel=self.voxels), int(nsteps),
                                ctypes.byref(p), _stream_handle(stream)), "evx_rd_step")
        return c

    def advance_record(self, nsteps: int, params: CHParams, traj: torch.Tensor, stream=None):
        """Advance nsteps, writing c^n at the start of each step to traj[n] (float32 device tensor
        of shape (>= nsteps, nz, ny, nx))."""
        p = params.c()
        ptr = None
        if nsteps > 0:
            if traj.numel() < nsteps * self.voxels:
                raise ValueError(f"traj holds {traj.numel()} values, needs {nsteps * self.voxels}")
            ptr = _dev_ptr(traj)
        _check(_LIB.evx_ch_advance_record(self._h, int(nsteps), ctypes.byref(p), ptr,
                                          _stream_handle(stream)), "evx_ch_advance_record")
        return traj

    def end(self, c: torch.Tensor, stream=None):
        _check(_LIB.evx_ch_end(self._h, _dev_ptr(c, numel=self.voxels), _stream_handle(stream)),
               "evx_ch_end")
        return c

    def restore(self, stream=None):
        _check(_LIB.evx_ch_restore(self._h, _stream_handle(stream)), "evx_ch_restore")

    def state(self) -> torch.Tensor:
        """The spectral state S as a uint8 view of the workspace (for checkpoint/resume)."""
        ptr, nb = ctypes.c_void_p(), ctypes.c_size_t()
        _check(_LIB.evx_plan_state(self._h, ctypes.byref(ptr), ctypes.byref(nb)), "evx_plan_state")
        off = ptr.value - self.workspace.data_ptr()
        return self.workspace[off:off + nb.value]

    # ------------------------------------------------------------------ adjoint, diagnostics
    def adjoint_step(self, c_n: torch.Tensor, lam: torch.Tensor, params: CHParams,
                     dkappa: torch.Tensor, dM: torch.Tensor, stream=None):
        """lam <- dL/dc^n from dL/dc^{n+1}; dkappa, dM (1-element float64 device tensors)
        accumulate the parameter gradients of this step."""
        p = params.c()
        _check(_LIB.evx_ch_adjoint_step(
            self._h, _dev_ptr(c_n, numel=self.voxels), _dev_ptr(lam, numel=self.voxels),
            ctypes.byref(p), _dev_ptr(dkappa, torch.float64, 1), _dev_ptr(dM, torch.float64, 1),
            _stream_handle(stream)), "evx_ch_adjoint_step")
        return lam

    def adjoint_sweep(self, states: torch.Tensor, nsteps: int, lam: torch.Tensor,
                      params: CHParams, dkappa: torch.Tensor, dM: torch.Tensor, stream=None):
        """nsteps adjoint steps backwards through states[0 .. nsteps-1] (c^0 .. c^{nsteps-1},
        the leading nsteps fields of a contiguous float32 tensor): lam <- dL/dc^0 from
        dL/dc^{nsteps}; dkappa, dM accumulate.  Bitwise equal to nsteps adjoint_step calls."""
        p = params.c()
        if states.numel() < nsteps * self.voxels:
            raise ValueError(f"states holds fewer than {nsteps} fields")
        _check(_LIB.evx_ch_adjoint_sweep(
            self._h, _dev_ptr(states), int(nsteps), _dev_ptr(lam, numel=self.voxels),
            ctypes.byref(p), _dev_ptr(dkappa, torch.float64, 1), _dev_ptr(dM, torch.float64, 1),
            _stream_handle(stream)), "evx_ch_adjoint_sweep")
        return lam

    def diagnostics(self, c: torch.Tensor, params: CHParams, out: torch.Tensor = None,
                    stream=None) -> torch.Tensor:
        """(mass, energy) of the real field c as a 2-element float64 device tensor."""
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=c.device)
        p = params.c()
        _check(_LIB.evx_ch_diagnostics(self._h, _dev_ptr(c, numel=self.voxels), ctypes.byref(p),
                                       _dev_ptr(out, torch.float64, 2), _stream_handle(stream)),
               "evx_ch_diagnostics")
        return out

    def distance(self, a: torch.Tensor, b: torch.Tensor, out: torch.Tensor = None,
                 stream=None) -> torch.Tensor:
        """(sum (a-b)^2, sum b^2) as a 2-element float64 device tensor."""
        if out is None:
            out = torch.empty(2, dtype=torch.float64, device=a.device)
        _check(_LIB.evx_ch_distance(self._h, _dev_ptr(a, numel=self.voxels),
                                    _dev_ptr(b, numel=self.voxels),
                                    _dev_ptr(out, torch.float64, 2), _stream_handle(stream)),
               "evx_ch_distance")
        return out

    # ------------------------------------------------------------------ measurement
    def enable_pass_timing(self, on: bool = True):
        _check(_LIB.evx_plan_enable_pass_timing(self._h, int(bool(on))),
               "evx_plan_enable_pass_timing")

    def read_pass_times(self):
        ms = (ctypes.c_double * 4)()
        cnt = (ctypes.c_longlong * 4)()
        _check(_LIB.evx_plan_read_pass_times(self._h, ms, cnt), "evx_plan_read_pass_times")
        return list(ms), list(cnt)

    def set_xcd_remap(self, on: bool):
        _check(_LIB.evx_plan_set_xcd_remap(self._h, int(bool(on))), "evx_plan_set_xcd_remap")

    def set_plane_pass(self, on: bool):
        """Run the step's y, x, y transforms as one launch per z plane where the grid allows
        (periodic, nx = ny = 32 or 64; the default), or always as three passes."""
        _check(_LIB.evx_plan_set_plane_pass(self._h, int(bool(on))), "evx_plan_set_plane_pass")

    def set_step_graph(self, steps: int):
        """Step-loop launch mode: chunks of `steps` steps replayed as one HIP graph (> 0), every
        kernel launched individually (0), or automatic (-1, the default)."""
        _check(_LIB.evx_plan_set_step_graph(self._h, int(steps)), "evx_plan_set_step_graph")
