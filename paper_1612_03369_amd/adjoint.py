"""``torch.autograd.Function`` over the multi-step advection map U -> x(T).

forward(U): set the nodal field, re-seed the store from the problem's initial
state, run ``pic_advance_checkpointed`` (checkpoints every k steps) and return
the final locations indexed by particle id ([dim][n_seeded], NaN for lost
particles).  backward(dL/dx): hand dL/dx in the store's order to
``pic_adjoint``, which re-runs each checkpoint segment and sweeps the RK
stages in reverse on the GPU, scatter-adding into dL/dU with FP64 atomics.
The Python side only converts between id order and store order.
"""
from __future__ import annotations

import torch

from . import _lib as L


class ParticleFlow:
    """Initial particle state + run parameters of one differentiable problem."""

    def __init__(self, problem, counts, xr, ids, dt, n_steps, scheme=L.PIC_RK4, ckpt_every=10):
        self.p = problem
        self.counts, self.xr, self.ids = counts, xr, ids
        self.n0 = int(xr.shape[1])
        self.dt, self.n_steps, self.scheme, self.ckpt = float(dt), int(n_steps), int(scheme), int(ckpt_every)
        self.ws = problem.adjoint_workspace(self.n_steps, self.ckpt)
        self.runs = 0           # forward runs so far: the store and checkpoints hold the last one

    def run_forward(self, U, checkpoint=True):
        p = self.p
        self.runs += 1
        p.set_velocity(U)
        p.seed_reference(self.counts, self.xr, self.ids)
        if checkpoint:
            p.advance_checkpointed(self.dt, self.n_steps, self.scheme, self.ckpt, self.ws)
        else:
            p.advance(self.dt, self.n_steps, self.scheme, L.PIC_F64)
        cur = p.current(copy=False)
        ids = cur["id"].long()
        out = torch.full((p.dim, self.n0), float("nan"), dtype=torch.float64, device=p.device)
        out[:, ids] = cur["x"]
        return out, ids


class _Advect(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, flow):
        out, ids = flow.run_forward(U.detach(), checkpoint=True)
        ctx.flow = flow
        ctx.ids = ids
        ctx.run = flow.runs
        ctx.shape = tuple(U.shape)
        ctx.save_for_backward(U)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        flow = ctx.flow
        p = flow.p
        if flow.runs != ctx.run:
            # another forward ran since: the store and the checkpoints belong to it, so this
            # forward is run again from its own field before the reverse sweep
            (U,) = ctx.saved_tensors
            _, ids = flow.run_forward(U.detach(), checkpoint=True)
            if not torch.equal(ids, ctx.ids):
                raise RuntimeError("re-run of the forward gave a different particle set")
            ctx.run = flow.runs
        cap = p.store.capacity
        dl = torch.zeros((p.dim, cap), dtype=torch.float64, device=p.device)
        n = ctx.ids.numel()
        g = grad_out.to(torch.float64)[:, ctx.ids]
        dl[:, :n] = torch.nan_to_num(g, nan=0.0)
        dU = torch.zeros(ctx.shape, dtype=torch.float64, device=p.device)
        p.adjoint(dl, flow.ws, dU)
        return dU, None


def advect(U: torch.Tensor, flow: ParticleFlow) -> torch.Tensor:
    """Final particle locations [dim][n_seeded] as a differentiable function of U."""
    return _Advect.apply(U, flow)
