"""torch.autograd wrapper of the integrator with step checkpointing.

trajectory(ctx, xm0, v0, nsteps, every, thr) returns the state after nsteps steps and records
the state every `every` steps. Backward walks the segments in reverse; each segment recomputes
its own states from its checkpoint inside the library (bit-identical to the forward run) and
applies the hand-written reverse-mode kernels of kick, jump and drift. Gradients flow to the
initial positions, velocities and masses (column 3 of xm); the critical radii are held fixed.
Memory: one (xm, v) pair per checkpoint plus 2 * every * n * 32 bytes of library workspace.
"""
from __future__ import annotations

import torch


class _Trajectory(torch.autograd.Function):
    @staticmethod
    def forward(fctx, xm0, v0, nb_ctx, thr, nsteps, every):
        xm = xm0.detach().clone().contiguous()
        v = v0.detach().clone().contiguous()
        checkpoints = []
        done = 0
        while done < nsteps:
            k = min(every, nsteps - done)
            checkpoints.append((xm.clone(), v.clone(), k))
            nb_ctx.step(xm, v, k, thr=thr)
            done += k
        fctx.checkpoints = checkpoints
        fctx.nb_ctx = nb_ctx
        fctx.thr = thr
        return xm, v

    @staticmethod
    def backward(fctx, gxm, gv):
        ref = fctx.checkpoints[0][0] if fctx.checkpoints else None
        lam_x = torch.zeros_like(ref) if gxm is None else gxm.detach().clone().contiguous()
        lam_v = torch.zeros_like(ref) if gv is None else gv.detach().clone().contiguous()
        for xm_c, v_c, k in reversed(fctx.checkpoints):
            fctx.nb_ctx.step_vjp(xm_c, v_c, fctx.thr, k, lam_x, lam_v)
        return lam_x, lam_v, None, None, None, None


def trajectory(nb_ctx, xm0, v0, nsteps, every=10, thr=None):
    """Differentiable nsteps-step integration. thr defaults to the thresholds of (xm0, v0)."""
    if thr is None:
        thr = nb_ctx.rcrit(xm0.detach().contiguous(), v0.detach().contiguous())
    return _Trajectory.apply(xm0, v0, nb_ctx, thr, int(nsteps), int(every))
