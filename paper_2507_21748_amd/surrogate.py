"""Learned coarse stepper: Python binding of the library's residual CNN (evx_surrogate_*), its
training on trajectories the solver itself generates, and a rollout controller that judges every
prediction with the solver and falls back to it.

Argument marshalling and control flow only; every array operation runs in the library's HIP
kernels (network, solver, diagnostics) except small host-side decisions on scalars.
"""
from __future__ import annotations

import ctypes
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import evx
from .inputs import quench_field, surrogate_init

__all__ = ["Net", "RolloutConfig", "rollout", "make_pairs", "sample_windows"]

_NET_PROTOS = {
    "evx_surrogate_param_count": [ctypes.POINTER(ctypes.c_size_t)],
    "evx_surrogate_create": [ctypes.POINTER(ctypes.c_void_p)],
    "evx_surrogate_destroy": [ctypes.c_void_p],
    "evx_surrogate_set_params": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "evx_surrogate_workspace_bytes": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_size_t)],
    "evx_surrogate_infer": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                            ctypes.c_size_t, ctypes.c_void_p],
    "evx_surrogate_train_step": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "evx_surrogate_train_buffers": [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_void_p)],
}
_BOUND = False


def _lib():
    global _BOUND
    lib = evx.load()
    if not _BOUND:
        for name, args in _NET_PROTOS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        _BOUND = True
    return lib


class _Workspace:
    def __init__(self, nbytes: int, device):
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self.off = (-self.buf.data_ptr()) % 256
        self.nbytes = nbytes

    @property
    def ptr(self):
        return ctypes.c_void_p(self.buf.data_ptr() + self.off)

    def view(self, dev_ptr: int, nbytes: int) -> torch.Tensor:
        o = dev_ptr - self.buf.data_ptr()
        return self.buf[o:o + nbytes]


class Net:
    """The coarse-stepper network with FP32 master parameters and Adam state on the device."""

    def __init__(self, params=None, seed: int = 0, device=None):
        lib = _lib()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None
                                   else device)
        n = ctypes.c_size_t()
        evx._check(lib.evx_surrogate_param_count(ctypes.byref(n)), "evx_surrogate_param_count")
        self.nparam = n.value
        if params is None:
            params = surrogate_init(seed)
        self.params = torch.as_tensor(np.asarray(params, np.float32)).to(self.device).contiguous()
        assert self.params.numel() == self.nparam
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            evx._check(lib.evx_surrogate_create(ctypes.byref(h)), "evx_surrogate_create")
        self._h = h
        self._ws = {}
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.set_params(self.params)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and evx._LIB is not None:
            evx._LIB.evx_surrogate_destroy(h)
            self._h = None

    def set_params(self, params: torch.Tensor):
        if params is not self.params:
            self.params.copy_(params)
        evx._check(evx._LIB.evx_surrogate_set_params(self._h, ctypes.c_void_p(self.params.data_ptr()),
                                                     evx._stream_handle()),
                   "evx_surrogate_set_params")

    def _workspace(self, shape, train: bool) -> _Workspace:
        key = (tuple(shape), train)
        if key not in self._ws:
            nz, ny, nx = shape
            nb = ctypes.c_size_t()
            evx._check(evx._LIB.evx_surrogate_workspace_bytes(nx, ny, nz, int(train),
                                                              ctypes.byref(nb)),
                       "evx_surrogate_workspace_bytes")
            self._ws[key] = _Workspace(nb.value, self.device)
        return self._ws[key]

    def release_workspaces(self):
        self._ws.clear()

    def infer(self, c: torch.Tensor, out: torch.Tensor = None,
              conserve_mass: bool = False) -> torch.Tensor:
        """out <- c + net(c) on the periodic grid of c (nz, ny, nx); with conserve_mass the
        increment's mean is removed."""
        nz, ny, nx = c.shape
        out = torch.empty_like(c) if out is None else out
        ws = self._workspace(c.shape, False)
        evx._check(evx._LIB.evx_surrogate_infer(
            self._h, evx._dev_ptr(c), evx._dev_ptr(out, numel=c.numel()), nx, ny, nz,
            int(bool(conserve_mass)), ws.ptr, ws.nbytes, evx._stream_handle()),
            "evx_surrogate_infer")
        return out

    def train_step(self, x: torch.Tensor, y: torch.Tensor, halo: int, lr: float) -> torch.Tensor:
        """One Adam step on windows x -> y of shape (batch, n, n, n); returns the loss (device
        float64 tensor) at the parameters before the update."""
        b, n = x.shape[0], x.shape[1]
        assert x.shape == (b, n, n, n) and y.shape == x.shape
        ws = self._workspace((n, n, n), True)
        self.step += 1
        evx._check(evx._LIB.evx_surrogate_train_step(
            self._h, evx._dev_ptr(x), evx._dev_ptr(y), b, n, halo,
            evx._dev_ptr(self.params), evx._dev_ptr(self.m), evx._dev_ptr(self.v), self.step,
            float(lr), evx._dev_ptr(self.loss, torch.float64, 1), ws.ptr, ws.nbytes,
            evx._stream_handle()), "evx_surrogate_train_step")
        return self.loss

    def train_buffers(self, n: int) -> dict:
        """Views of the last train step's stored activations and gradients (verification)."""
        ws = self._workspace((n, n, n), True)
        ptrs = (ctypes.c_void_p * 13)()
        evx._check(evx._LIB.evx_surrogate_train_buffers(ws.ptr, ws.nbytes, n, ptrs),
                   "evx_surrogate_train_buffers")
        V = n ** 3

        def bf(i, ch):
            return ws.view(ptrs[i], V * ch * 2).view(torch.bfloat16).reshape(n, n, n, ch)

        def f32(i, count):
            return ws.view(ptrs[i], count * 4).view(torch.float32)

        return {"x0": bf(0, 1)[..., 0], "z1": bf(1, 32), "a1": bf(2, 32), "z2": bf(3, 32),
                "a2": bf(4, 32), "z3": bf(5, 32), "a3": bf(6, 32), "dz1": bf(7, 32),
                "dz2": bf(8, 32), "dz3": bf(9, 32), "out": f32(10, V).reshape(n, n, n),
                "dy": f32(11, V).reshape(n, n, n), "grads": f32(12, self.nparam)}


# ------------------------------------------------------------------------------ training data
def make_pairs(shape, means, seeds, nsteps: int, stride: int, every: int, params: "evx.CHParams",
               bc="periodic", scheme="spectral"):
    """Solver trajectories from seeded quenches: for each (mean, seed) a run of nsteps steps;
    returns a list of (c_n, c_{n+stride}) device pairs for n = 0, every, 2 every, ..."""
    pairs = []
    plan = evx.Plan(shape, bc, scheme)
    for mean in means:
        for seed in seeds:
            c = torch.from_numpy(quench_field(shape, mean, 0.05, seed)).cuda()
            plan.begin(c)
            snaps = {}
            for n in range(0, nsteps + 1, every):
                if n > 0:
                    plan.advance(every, params)
                out = torch.empty_like(c)
                plan.end(out)
                snaps[n] = out
            for n in snaps:
                if n + stride in snaps:
                    pairs.append((snaps[n], snaps[n + stride]))
    return pairs


def sample_windows(pairs, batch: int, edge: int, rng: np.random.Generator):
    """Random edge^3 windows (periodic wrap) of random pairs: (x, y) of shape (batch, e, e, e)."""
    xs, ys = [], []
    for _ in range(batch):
        a, b = pairs[int(rng.integers(len(pairs)))]
        nz, ny, nx = a.shape
        o = [int(rng.integers(s)) for s in (nz, ny, nx)]
        idx = [torch.arange(o[k], o[k] + edge, device=a.device) % a.shape[k] for k in range(3)]
        xs.append(a[idx[0]][:, idx[1]][:, :, idx[2]])
        ys.append(b[idx[0]][:, idx[1]][:, :, idx[2]])
    return torch.stack(xs).contiguous(), torch.stack(ys).contiguous()


# ------------------------------------------------------------------------------ rollout
@dataclass
class RolloutConfig:
    """How the solver judges the network.

    Every prediction must keep the mass (|d mean| <= mass_tol) and must not raise the free energy
    (E_new <= E (1 + energy_rtol)); a prediction failing either is replaced by the solver.  Spot
    checks compare predictions with the solver's own `stride` steps at relative L2 <= spot_tol,
    in one of two modes:

    verify = "window": a check covers the checked application alone, from its own start state.
      Checks are drawn at random (rate 1 / check_every, seeded), and the last application is
      always checked.  After a failed check every application is checked until one passes, so
      a failing network never runs unverified.  The applications between checks are accepted on
      mass and energy alone, which a wrong prediction can pass: fast, but the error of an
      unchecked window is not bounded.
    verify = "span": a check runs the solver from the last verified state over every application
      since (at most check_every of them, and at the end), compares the final states, and on a
      failure replaces the whole span by the solver's result.  Every state the rollout hands on
      at a check is then within spot_tol of the solver started from the previous verified state,
      whatever the network does between checks -- but the solver runs over every window, so the
      rollout costs at least the plain solver's time.
    """
    stride: int = 10             # solver steps replaced by one network application
    check_every: int = 10        # mean applications per spot check
    mass_tol: float = 1e-5       # |mean(c_new) - mean(c)| allowed per application
    energy_rtol: float = 1e-6    # E(c_new) <= E(c) (1 + energy_rtol)
    spot_tol: float = 2e-3       # relative L2 to the solver on a spot check
    conserve_mass: bool = True   # remove the mean of every predicted increment
    verify: str = "span"         # "span" (sound) or "window" (fast; see above)
    seed: int = 0                # draws of the checked windows


@dataclass
class RolloutStats:
    applications: int = 0
    accepted: int = 0            # predictions the rollout kept
    fallback_mass: int = 0
    fallback_energy: int = 0
    fallback_spot: int = 0       # failed spot checks (their window or span was recomputed)
    spot_checks: int = 0
    solver_windows: int = 0      # windows of `stride` solver steps run (checks and fallbacks)
    spot_errors: list = field(default_factory=list)
    seconds: float = 0.0


def rollout(net: Net, c0: torch.Tensor, napps: int, params: "evx.CHParams",
            cfg: RolloutConfig = RolloutConfig(), plan: "evx.Plan" = None):
    """napps coarse steps of `stride` solver steps each from c0 (periodic spectral grid), every
    prediction judged by the solver (mass, energy, spot checks; see RolloutConfig) and replaced by
    it when rejected.  Returns (c, stats)."""
    if cfg.verify not in ("window", "span"):
        raise ValueError(f"unknown verify mode {cfg.verify!r}")
    shape = tuple(c0.shape)
    if plan is None:
        plan = evx.Plan(shape, "periodic", "spectral", ops=evx.OP_STEP | evx.OP_DIAG)
    V = c0.numel()
    rng = np.random.default_rng(cfg.seed)
    st = RolloutStats()
    c = c0.clone()
    cand = torch.empty_like(c)
    diag = torch.empty(2, dtype=torch.float64, device=c.device)
    sync = torch.cuda.synchronize if c.is_cuda else (lambda: None)

    def solve(start, windows):
        out = start.clone()
        plan.step(out, windows * cfg.stride, params)
        st.solver_windows += windows
        return out

    def rel_err(a, b):
        dd = plan.distance(a, b, out=diag).cpu().numpy()
        return float(np.sqrt(dd[0] / dd[1]))

    sync()
    t0 = time.perf_counter()
    d_cur = plan.diagnostics(c, params).cpu().numpy()
    strict = True                     # window mode: check until a prediction passes
    anchor, span = c.clone(), 0       # span mode: last verified state, windows since
    for k in range(napps):
        st.applications += 1
        last = k == napps - 1
        net.infer(c, cand, conserve_mass=cfg.conserve_mass)
        d_new = plan.diagnostics(cand, params, out=diag).cpu().numpy()
        ok = True
        if abs(d_new[0] - d_cur[0]) / V > cfg.mass_tol:
            st.fallback_mass += 1
            ok = False
        elif d_new[1] > d_cur[1] * (1 + cfg.energy_rtol):
            st.fallback_energy += 1
            ok = False
        if cfg.verify == "window":
            ref = None
            if ok and (strict or last or rng.random() < 1.0 / max(cfg.check_every, 1)):
                ref = solve(c, 1)
                err = rel_err(cand, ref)
                st.spot_checks += 1
                st.spot_errors.append(err)
                if err > cfg.spot_tol:
                    st.fallback_spot += 1
                    ok = False
                strict = not ok
            if ok:
                st.accepted += 1
                c, cand = cand, c
                d_cur = d_new
            else:
                c = ref if ref is not None else solve(c, 1)
                d_cur = plan.diagnostics(c, params).cpu().numpy()
            continue
        # span mode
        span += 1
        if not ok:                    # the span's earlier, unverified windows are redone too
            c = solve(anchor, span)
            anchor, span = c.clone(), 0
            d_cur = plan.diagnostics(c, params).cpu().numpy()
            continue
        if span >= cfg.check_every or last:
            ref = solve(anchor, span)
            err = rel_err(cand, ref)
            st.spot_checks += 1
            st.spot_errors.append(err)
            if err > cfg.spot_tol:
                st.fallback_spot += 1
                c = ref
                d_cur = plan.diagnostics(c, params).cpu().numpy()
            else:
                st.accepted += span
                c, cand = cand, c
                d_cur = d_new
            anchor, span = c.clone(), 0
            continue
        c, cand = cand, c             # provisional until the span's check
        d_cur = d_new
    sync()
    st.seconds = time.perf_counter() - t0
    return c, st
