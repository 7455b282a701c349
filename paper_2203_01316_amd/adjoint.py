"""Gradients of objectives of the advection-diffusion lattice with respect to
its source field, as torch.autograd.Functions over liblbm.so: a final-state
objective (SourceObjective) and an objective summed over observation times
(TrackingObjective, whose reverse sweep replays the checkpointed forward).

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


class TrackingObjective(torch.autograd.Function):
    """J = sum over the observation times t = every, 2 every, ..., <= steps of
    1/2 sum (H_t - H*_t)^2.  Its reverse sweep needs the residual of every
    observation time, which depends on the forward state at that time: with
    recompute=True the forward keeps a raw snapshot every `interval` steps and
    the backward replays each segment from its snapshot to recompute them
    (memory: about T / interval snapshots plus one segment's residuals); with
    recompute=False the forward keeps every residual."""

    @staticmethod
    def forward(ctx, Qsrc, model, H0, targets, steps, every, interval, recompute):
        model.set_source(Qsrc.detach())
        model.init(H0)
        obs = list(range(every, steps + 1, every))
        tgt = _targets(model, targets, len(obs))
        snaps, resid = {}, {}
        J = 0.0
        for t in range(steps):
            if recompute and t % interval == 0:
                snaps[t] = model.save_state()
            model.step(1)
            if (t + 1) % every == 0:
                Jt, r = model.objective_residual(tgt[(t + 1) // every - 1])
                J += Jt
                if not recompute or t + 1 == steps:
                    resid[t + 1] = r
        ctx.model, ctx.snaps, ctx.resid, ctx.tgt = model, snaps, resid, tgt
        ctx.steps, ctx.every, ctx.interval, ctx.recompute = steps, every, interval, recompute
        ctx.qdtype = Qsrc.dtype
        return torch.tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        model, steps, every = ctx.model, ctx.steps, ctx.every
        lam = torch.zeros(model.Q, model.n, dtype=model.rdtype, device=model.device)
        other = torch.empty_like(lam)
        dq = torch.zeros(model.n, dtype=torch.float64, device=model.device)
        if steps % every == 0:
            model.adjoint_seed(ctx.resid.pop(steps), lam, dq, accumulate=True)
        starts = list(range(0, steps, ctx.interval))
        for s0 in reversed(starts):
            s1 = min(s0 + ctx.interval, steps)
            seg = {}
            if ctx.recompute:
                # forward states s0 .. s1 - 1 of the segment, from its snapshot
                model.load_state(ctx.snaps.pop(s0))
                for t in range(s0, s1):
                    if t > 0 and t % every == 0:
                        seg[t] = model.objective_residual(ctx.tgt[t // every - 1])[1]
                    if t + 1 < s1:
                        model.step(1)
            else:
                seg = {t: ctx.resid.pop(t) for t in range(max(s0, 1), s1) if t % every == 0}
            for t in range(s1 - 1, s0 - 1, -1):
                model.adjoint_step(lam, other, dq)
                lam, other = other, lam
                if t in seg:
                    model.adjoint_seed(seg.pop(t), lam, dq, accumulate=True)
        model.sync()
        grad = dq * gJ.to(dq.device, torch.float64)
        ctx.model = ctx.snaps = ctx.resid = ctx.tgt = None
        return grad.to(ctx.qdtype), None, None, None, None, None, None, None


def _targets(model, targets, nobs):
    """One FP64 device target per observation time: `targets` is one array for
    every time or a sequence of nobs arrays."""
    torch = model.torch
    if isinstance(targets, (list, tuple)):
        assert len(targets) == nobs, f"{len(targets)} targets for {nobs} observation times"
        return [torch.as_tensor(t, dtype=torch.float64, device=model.device).reshape(model.n) for t in targets]
    one = torch.as_tensor(targets, dtype=torch.float64, device=model.device).reshape(model.n)
    return [one] * nobs


def tracking_objective(Qsrc, model: "L.LBM", H0, targets, steps: int, every: int = 1, interval: int | None = None,
                       recompute: bool = True):
    """J(Q) = sum over t = every, 2 every, ... <= steps of 1/2 sum (H_t - H*_t)^2
    for the context `model` (advection-only, with_source=1); differentiable
    with respect to Qsrc.  targets: one array for every observation time or
    one per time."""
    if interval is None:
        interval = max(1, int(math.ceil(math.sqrt(steps))))
    assert steps >= 1 and every >= 1
    return TrackingObjective.apply(Qsrc, model, H0, targets, int(steps), int(every), int(interval), bool(recompute))
