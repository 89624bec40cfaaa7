"""Differentiable Cahn-Hilliard rollout: gradients of any loss of c^T with respect to c^0, kappa
and M through the library's hand-written adjoint steps (evx_ch_adjoint_sweep).

Memory, two modes:
  every > 0: the forward pass keeps the spectral state every `every` steps (8 bytes per voxel
    each); the backward pass recomputes one segment at a time from its checkpoint (bit-identical
    to the forward trajectory, since every kernel rounds deterministically) and sweeps it
    backwards, holding `every` real fields.
  every = 0: the forward pass records every state it passes through (4 bytes per voxel per step:
    1.7 GB for 200 steps of 128^3) and the backward pass sweeps them without recomputation.
Both give bitwise the same gradients.
"""
from __future__ import annotations

import torch

from . import evx

__all__ = ["CHRollout", "ch_rollout"]


class CHRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c0, kappa, M, plan, nsteps, dt, A, every):
        if nsteps < 1 or every < 0:
            raise ValueError("nsteps must be >= 1 and every >= 0")
        prm = evx.CHParams(dt=float(dt), M=float(M.item()), kappa=float(kappa.item()), A=float(A))
        c = c0.detach().to(torch.float32).contiguous().clone()
        plan.begin(c)
        ckpts, traj = [], None
        if every == 0:
            traj = torch.empty((nsteps,) + tuple(c.shape), dtype=torch.float32, device=c.device)
            plan.advance_record(nsteps, prm, traj)
        else:
            for s in range(0, nsteps, every):
                ckpts.append(plan.state().clone())
                plan.advance(min(every, nsteps - s), prm)
        cT = torch.empty_like(c)
        plan.end(cT)
        ctx.plan, ctx.prm, ctx.nsteps, ctx.every, ctx.ckpts = plan, prm, nsteps, every, ckpts
        ctx.traj = traj
        ctx.kappa_meta = (kappa.dtype, kappa.device, kappa.shape)
        ctx.M_meta = (M.dtype, M.device, M.shape)
        return cT

    @staticmethod
    def backward(ctx, grad_cT):
        plan, prm, nsteps, every = ctx.plan, ctx.prm, ctx.nsteps, ctx.every
        lam = grad_cT.detach().to(torch.float32).contiguous().clone()
        dk = torch.zeros(1, dtype=torch.float64, device=lam.device)
        dM = torch.zeros(1, dtype=torch.float64, device=lam.device)
        if ctx.traj is not None:
            plan.adjoint_sweep(ctx.traj, nsteps, lam, prm, dk, dM)
        else:
            # one buffer for every segment's states (the first segment is the longest)
            states = torch.empty((min(every, nsteps),) + tuple(lam.shape), dtype=torch.float32,
                                 device=lam.device)
            for seg in range(len(ctx.ckpts) - 1, -1, -1):
                k = min(every, nsteps - seg * every)
                plan.state().copy_(ctx.ckpts[seg])
                plan.restore()
                # c^n of the segment: k - 1 recorded steps, then the last state
                plan.advance_record(k - 1, prm, states)
                plan.end(states[k - 1])
                plan.adjoint_sweep(states, k, lam, prm, dk, dM)
            del states
        ctx.ckpts, ctx.traj = None, None
        kd, kdev, kshape = ctx.kappa_meta
        md, mdev, mshape = ctx.M_meta
        return (lam, dk.to(kd).to(kdev).reshape(kshape), dM.to(md).to(mdev).reshape(mshape),
                None, None, None, None, None)


def ch_rollout(c0: torch.Tensor, kappa: torch.Tensor, M: torch.Tensor, plan: "evx.Plan",
               nsteps: int, dt: float, A: float = 2.0, every: int = 20) -> torch.Tensor:
    """c^T after nsteps steps from c0, differentiable w.r.t. c0, kappa and M (0-d tensors).
    The plan must have been created with ops including evx.OP_ADJOINT.  every > 0: spectral
    checkpoints every `every` steps, segments recomputed in the backward pass; every = 0: every
    state recorded in the forward pass (nsteps real fields of device memory)."""
    return CHRollout.apply(c0, kappa, M, plan, int(nsteps), float(dt), float(A), int(every))
