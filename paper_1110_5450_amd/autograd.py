"""Differentiable sweep: torch.autograd.Function over the C ABI.

forward  -> sweep_eval_batched (positions and normals),
backward -> sweep_backward_ex (hand-written adjoint kernels) with the
incoming gradients of positions and normals, giving dL/d(path control
points) and dL/d(profile control points) in float64.

Each call works on its own shallow copy of the caller's Batch (the caller's
object is never modified), and the control-point tensors are kept with
save_for_backward, so two forward calls on one Batch each differentiate their
own control points, and an in-place change of them before backward raises.
"""

from __future__ import annotations

import copy
from typing import Optional

import torch

from . import api


def _with_ctrl(batch: api.Batch, path_ctrl: torch.Tensor, prof_ctrl: torch.Tensor) -> api.Batch:
    b = copy.copy(batch)
    b.path_ctrl = path_ctrl.detach().contiguous()
    b.prof_ctrl = prof_ctrl.detach().contiguous()
    return b


class SweepFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, path_ctrl: torch.Tensor, prof_ctrl: torch.Tensor, batch: api.Batch, out_dtype, initial_normal):
        ctx.set_materialize_grads(False)
        pos, nrm = api.sweep_eval_batched(_with_ctrl(batch, path_ctrl, prof_ctrl), out_dtype=out_dtype,
                                          initial_normal=initial_normal)
        ctx.save_for_backward(path_ctrl, prof_ctrl)
        ctx.batch = batch
        ctx.initial_normal = initial_normal
        return pos, nrm

    @staticmethod
    def backward(ctx, grad_pos: Optional[torch.Tensor], grad_nrm: Optional[torch.Tensor]):
        if grad_pos is None and grad_nrm is None:
            return None, None, None, None, None
        path_ctrl, prof_ctrl = ctx.saved_tensors
        gP, gQ = api.sweep_backward(_with_ctrl(ctx.batch, path_ctrl, prof_ctrl), grad_pos, grad_nrm=grad_nrm,
                                    initial_normal=ctx.initial_normal)
        return gP, gQ, None, None, None


def sweep(path_ctrl: torch.Tensor, prof_ctrl: torch.Tensor, batch: api.Batch, out_dtype=torch.float32,
          initial_normal=None):
    """Differentiable batched sweep: returns flat (positions, normals); use
    batch.view(flat, k) for sweep k's (3, n_u, n_v) block.  path_ctrl and
    prof_ctrl are the packed (sum n, 3) float64 device tensors; batch gives
    the counts, degrees, knots, weights and grid sizes (its own control-point
    tensors are not used and not modified)."""
    return SweepFunction.apply(path_ctrl, prof_ctrl, batch, out_dtype, initial_normal)
