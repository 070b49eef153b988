"""Autograd wrappers of the upsampling step and of checkpointed rollouts.

``UpsampleStep`` differentiates one step through the library's adjoint
kernel; its forward records the per-particle sums the adjoint needs (a
"tape", upsample_step_taped).  ``UpsampleRollout`` advances the HR state
through a sequence of LR frames, keeping the state every ``checkpoint_every``
steps; its backward replays one segment at a time from its checkpoint
(recording tapes and saving each replayed step's LR grid, so that its
adjoint does not rebuild it) and runs the adjoint steps of that segment in
reverse, so
memory grows with T / checkpoint_every + the segment length instead of T.  Gradients reach the LR positions and velocities
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
        tape = torch.empty((6, hr_x.shape[1]), dtype=torch.float32, device=hr_x.device)
        x1, v1 = up.step(lr_x, lr_v, lr_rigid, hr_x, hr_v, tape=tape)
        ctx.up = up
        ctx.rigid = lr_rigid
        ctx.save_for_backward(lr_x, lr_v, hr_x, hr_v, tape)
        return x1, v1

    @staticmethod
    def backward(ctx, gx1, gv1):
        lr_x, lr_v, hr_x, hr_v, tape = ctx.saved_tensors
        gx1 = _zeros_like_or(gx1, hr_x)
        gv1 = _zeros_like_or(gv1, hr_v)
        gx, gv, glx, glv = ctx.up.step_backward(lr_x, lr_v, ctx.rigid, hr_x, hr_v, gx1, gv1, tape=tape)
        return None, glx, glv, gx, gv, None


def upsample_step(up: Upsampler, lr_x, lr_v, hr_x, hr_v, lr_rigid=None):
    return UpsampleStep.apply(up, lr_x, lr_v, hr_x, hr_v, lr_rigid)


class UpsampleRollout(torch.autograd.Function):
    """T steps against frames lr_x[t], lr_v[t] ([T, 3, N_L] each); returns the
    HR state after the last step, in the caller's particle order.

    With ``reorder`` the HR state is reordered spatially (upsample_sort_hr) at
    every checkpoint and every ``reorder_every`` steps, so the lanes of each
    wave stay neighbours as particles drift; per-particle results do not
    depend on the order.  The forward keeps each permutation: the reorders are
    undone on the output, the backward's segment replay applies the stored
    permutations (a fresh reorder could order equal keys differently), and
    gradients are mapped back through each of them (the adjoint of a gather
    is the scatter with the same permutation)."""

    @staticmethod
    def forward(ctx, up: Upsampler, checkpoint_every: int, reorder: bool, reorder_every: int, hr_x0, hr_v0,
                lr_x, lr_v, lr_rigid=None):
        T = lr_x.shape[0]
        every = max(1, int(checkpoint_every))
        re = max(1, int(reorder_every)) if reorder_every else every
        x, v = hr_x0.contiguous(), hr_v0.contiguous()
        perms = {}        # step t -> permutation applied to the state before step t
        checkpoints = []  # state before step seg * every (after its reorder)
        for t in range(T):
            if reorder and (t % every == 0 or t % re == 0):
                sx, sv = torch.empty_like(x), torch.empty_like(v)
                perms[t] = up.sort_hr(x, v, out_x=sx, out_v=sv)
                x, v = sx, sv
            if t % every == 0:
                checkpoints.append((x, v))
            x, v = up.step(lr_x[t], lr_v[t], lr_rigid, x, v)
        for t in sorted(perms, reverse=True):
            x, v = up.permute(x, perms[t], v, scatter=True)
        ctx.up, ctx.every, ctx.T, ctx.rigid = up, every, T, lr_rigid
        ctx.checkpoints, ctx.perms = checkpoints, perms
        ctx.save_for_backward(lr_x, lr_v)
        return x, v

    @staticmethod
    def backward(ctx, gxT, gvT):
        lr_x, lr_v = ctx.saved_tensors
        up, every, T, perms = ctx.up, ctx.every, ctx.T, ctx.perms
        gx = _zeros_like_or(gxT, ctx.checkpoints[0][0])
        gv = _zeros_like_or(gvT, ctx.checkpoints[0][1])
        # into the order of the final state
        for t in sorted(perms):
            gx, gv = up.permute(gx, perms[t], gv)
        g_lr_x = torch.zeros_like(lr_x)
        g_lr_v = torch.zeros_like(lr_v)
        for seg in range(len(ctx.checkpoints) - 1, -1, -1):
            start = seg * every
            end = min(start + every, T)
            # replay the segment from its checkpoint with the forward's
            # reorders, recording each replayed step's sums; the last step of
            # the segment is not replayed, its adjoint recomputes them
            states = [ctx.checkpoints[seg]]
            n = states[0][0].shape[1]
            k = max(end - start - 1, 1)
            tapes = torch.empty((k, 6, n), dtype=torch.float32, device=states[0][0].device)
            # each replayed step's LR grid, kept for its adjoint (no rebuild)
            grids = torch.empty((k, up.grid_snapshot_bytes()), dtype=torch.uint8, device=states[0][0].device)
            for t in range(start, end - 1):
                x, v = up.step(lr_x[t], lr_v[t], ctx.rigid, *states[-1], tape=tapes[t - start])
                up.grid_snapshot(grids[t - start])
                if t + 1 in perms:
                    x, v = up.permute(x, perms[t + 1], v)
                states.append((x, v))
            for t in range(end - 1, start - 1, -1):
                x, v = states[t - start]
                tape = tapes[t - start] if t < end - 1 else None
                grid = grids[t - start] if t < end - 1 else None
                gx, gv, _, _ = up.step_backward(lr_x[t], lr_v[t], ctx.rigid, x, v, gx, gv,
                                                g_lr_x=g_lr_x[t], g_lr_v=g_lr_v[t], tape=tape, grid=grid)
                if t in perms:
                    gx, gv = up.permute(gx, perms[t], gv, scatter=True)
        ctx.checkpoints = None
        ctx.perms = None
        return None, None, None, None, gx, gv, g_lr_x, g_lr_v, None


def rollout(up: Upsampler, hr_x0, hr_v0, lr_x, lr_v, checkpoint_every: int = 8, lr_rigid=None,
            reorder: bool = True, reorder_every: int = 0):
    """Checkpointed differentiable rollout; lr_x, lr_v: [T, 3, N_L].
    ``reorder_every`` (0: at checkpoints only) adds reorders inside segments."""
    return UpsampleRollout.apply(up, checkpoint_every, reorder, reorder_every, hr_x0, hr_v0, lr_x, lr_v, lr_rigid)
