"""Autograd wrappers of the upsampling step and of checkpointed rollouts.

``UpsampleStep`` differentiates one step through the library's adjoint
kernel.  ``UpsampleRollout`` advances the HR state through a sequence of LR
frames, keeping the state every ``checkpoint_every`` steps; its backward
replays one segment at a time from its checkpoint and runs the adjoint steps
of that segment in reverse, so memory grows with T / checkpoint_every + the
segment length instead of T.  Gradients reach the LR positions and velocities
of every frame and the initial HR state.  The LR simulation itself is not
differentiated (its frames are leaves).

All arithmetic runs in libupsample.so; this module only orders the calls.
"""
from __future__ import annotations

from typing import Optional

import torch

from .upsampler import Upsampler


def _zeros_like_or(t: Optional[torch.Tensor], like: torch.Tensor) -> torch.Tensor:
    return torch.zeros_like(like) if t is None else t.contiguous()


class UpsampleStep(torch.autograd.Function):
    """(lr_x, lr_v, hr_x, hr_v) -> (hr_x', hr_v') for one upsampling step."""

    @staticmethod
    def forward(ctx, up: Upsampler, lr_x, lr_v, hr_x, hr_v, lr_rigid=None):
        x1, v1 = up.step(lr_x, lr_v, lr_rigid, hr_x, hr_v)
        ctx.up = up
        ctx.rigid = lr_rigid
        ctx.save_for_backward(lr_x, lr_v, hr_x, hr_v)
        return x1, v1

    @staticmethod
    def backward(ctx, gx1, gv1):
        lr_x, lr_v, hr_x, hr_v = ctx.saved_tensors
        gx1 = _zeros_like_or(gx1, hr_x)
        gv1 = _zeros_like_or(gv1, hr_v)
        gx, gv, glx, glv = ctx.up.step_backward(lr_x, lr_v, ctx.rigid, hr_x, hr_v, gx1, gv1)
        return None, glx, glv, gx, gv, None


def upsample_step(up: Upsampler, lr_x, lr_v, hr_x, hr_v, lr_rigid=None):
    return UpsampleStep.apply(up, lr_x, lr_v, hr_x, hr_v, lr_rigid)


class UpsampleRollout(torch.autograd.Function):
    """T steps against frames lr_x[t], lr_v[t] ([T, 3, N_L] each); returns the
    HR state after the last step, in the caller's particle order.

    With ``reorder`` the HR state is reordered spatially (upsample_sort_hr) at
    every checkpoint, so the lanes of each wave stay neighbours as particles
    drift; per-particle results do not depend on the order, the reorders are
    undone on the output, and gradients are mapped back through each of them
    (the adjoint of a gather is the scatter with the same permutation)."""

    @staticmethod
    def forward(ctx, up: Upsampler, checkpoint_every: int, reorder: bool, hr_x0, hr_v0, lr_x, lr_v,
                lr_rigid=None):
        T = lr_x.shape[0]
        every = max(1, int(checkpoint_every))
        x, v = hr_x0.contiguous(), hr_v0.contiguous()
        checkpoints = []  # (x, v, perm applied before the segment or None)
        for t in range(T):
            if t % every == 0:
                perm = None
                if reorder:
                    sx, sv = torch.empty_like(x), torch.empty_like(v)
                    perm = up.sort_hr(x, v, out_x=sx, out_v=sv)
                    x, v = sx, sv
                checkpoints.append((x, v, perm))
            x, v = up.step(lr_x[t], lr_v[t], lr_rigid, x, v)
        for _, _, perm in reversed(checkpoints):
            if perm is not None:
                x, v = up.permute(x, perm, v, scatter=True)
        ctx.up, ctx.every, ctx.T, ctx.rigid = up, every, T, lr_rigid
        ctx.checkpoints = checkpoints
        ctx.save_for_backward(lr_x, lr_v)
        return x, v

    @staticmethod
    def backward(ctx, gxT, gvT):
        lr_x, lr_v = ctx.saved_tensors
        up, every, T = ctx.up, ctx.every, ctx.T
        gx = _zeros_like_or(gxT, ctx.checkpoints[0][0])
        gv = _zeros_like_or(gvT, ctx.checkpoints[0][1])
        # into the order of the last segment
        for _, _, perm in ctx.checkpoints:
            if perm is not None:
                gx, gv = up.permute(gx, perm, gv)
        g_lr_x = torch.zeros_like(lr_x)
        g_lr_v = torch.zeros_like(lr_v)
        for seg in range(len(ctx.checkpoints) - 1, -1, -1):
            start = seg * every
            end = min(start + every, T)
            # replay the segment from its checkpoint
            states = [ctx.checkpoints[seg][:2]]
            for t in range(start, end - 1):
                states.append(up.step(lr_x[t], lr_v[t], ctx.rigid, *states[-1]))
            for t in range(end - 1, start - 1, -1):
                x, v = states[t - start]
                gx, gv, _, _ = up.step_backward(lr_x[t], lr_v[t], ctx.rigid, x, v, gx, gv,
                                                g_lr_x=g_lr_x[t], g_lr_v=g_lr_v[t])
            perm = ctx.checkpoints[seg][2]
            if perm is not None:
                gx, gv = up.permute(gx, perm, gv, scatter=True)
        ctx.checkpoints = None
        return None, None, None, gx, gv, g_lr_x, g_lr_v, None


def rollout(up: Upsampler, hr_x0, hr_v0, lr_x, lr_v, checkpoint_every: int = 8, lr_rigid=None,
            reorder: bool = True):
    """Checkpointed differentiable rollout; lr_x, lr_v: [T, 3, N_L]."""
    return UpsampleRollout.apply(up, checkpoint_every, reorder, hr_x0, hr_v0, lr_x, lr_v, lr_rigid)
