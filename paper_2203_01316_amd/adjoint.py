"""Gradient of a final-state objective with respect to the source field of the
advection-diffusion lattice, as a torch.autograd.Function over liblbm.so.

Forward: T steps of the HIP step kernel with the source Q (App. D) as the
context's source field, then J = 1/2 sum (H_T - H*)^2 over the non-solid
nodes (lbm_objective).
Backward: T reverse steps of the HIP adjoint kernel (lbm_adjoint_step), the
exact transpose of the forward step, accumulating dJ/dQ.

Checkpointing: every `interval` steps (default ceil(sqrt(T))) the forward
stores a raw state snapshot (lbm_save_state).  With recompute=True the
backward walks the segments in reverse, restores each snapshot and replays the
segment before running its reverse steps: the schedule a reverse pass over a
nonlinear step needs.  The advection-diffusion step with a prescribed velocity
is affine in (state, Q), so its reverse step reads no forward state and
recompute=False gives the same gradient without the replay.
"""
from __future__ import annotations

import math

import torch

from . import lbm as L


class SourceObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Qsrc, model, H0, H_target, steps, interval, recompute):
        model.set_source(Qsrc.detach())
        model.init(H0)
        snaps = {}
        for t in range(steps):
            if recompute and t % interval == 0:
                snaps[t] = model.save_state()
            model.step(1)
        J, lam, dq = model.objective(H_target)
        ctx.model, ctx.lam, ctx.dq, ctx.snaps = model, lam, dq, snaps
        ctx.steps, ctx.interval, ctx.recompute = steps, interval, recompute
        ctx.qdtype = Qsrc.dtype
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        model, lam, dq = ctx.model, ctx.lam, ctx.dq
        other = torch.empty_like(lam)
        starts = list(range(0, ctx.steps, ctx.interval))
        for s0 in reversed(starts):
            s1 = min(s0 + ctx.interval, ctx.steps)
            if ctx.recompute:
                model.load_state(ctx.snaps.pop(s0))
                model.step(s1 - s0 - 1)  # forward states of the segment
            for _ in range(s1 - s0):
                model.adjoint_step(lam, other, dq)
                lam, other = other, lam
        model.sync()
        grad = dq * gJ.to(dq.device, torch.float64)
        ctx.model = ctx.lam = ctx.dq = ctx.snaps = None
        return grad.to(ctx.qdtype), None, None, None, None, None, None


def source_objective(Qsrc, model: "L.LBM", H0, H_target, steps: int, interval: int | None = None,
                     recompute: bool = True):
    """J(Q) for the context `model` (advection-only, periodic, with_source=1);
    differentiable with respect to Qsrc (a tensor on the model's device)."""
    if interval is None:
        interval = max(1, int(math.ceil(math.sqrt(steps))))
    return SourceObjective.apply(Qsrc, model, H0, H_target, int(steps), int(interval), bool(recompute))
