"""Differentiable sweep: torch.autograd.Function over the C ABI.

forward  -> sweep_eval_batched (positions and normals),
backward -> sweep_backward_ex (hand-written adjoint kernels) with the
incoming gradients of positions and normals, giving dL/d(path control
points) and dL/d(profile control points) in float64.
"""

from __future__ import annotations

from typing import Optional

import torch

from . import api


class SweepFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, path_ctrl: torch.Tensor, prof_ctrl: torch.Tensor, batch: api.Batch, out_dtype, initial_normal):
        ctx.set_materialize_grads(False)
        batch.path_ctrl = path_ctrl.detach().contiguous()
        batch.prof_ctrl = prof_ctrl.detach().contiguous()
        pos, nrm = api.sweep_eval_batched(batch, out_dtype=out_dtype, initial_normal=initial_normal)
        ctx.batch = batch
        ctx.initial_normal = initial_normal
        return pos, nrm

    @staticmethod
    def backward(ctx, grad_pos: Optional[torch.Tensor], grad_nrm: Optional[torch.Tensor]):
        if grad_pos is None and grad_nrm is None:
            return None, None, None, None, None
        gP, gQ = api.sweep_backward(ctx.batch, grad_pos, grad_nrm=grad_nrm, initial_normal=ctx.initial_normal)
        return gP, gQ, None, None, None


def sweep(path_ctrl: torch.Tensor, prof_ctrl: torch.Tensor, batch: api.Batch, out_dtype=torch.float32,
          initial_normal=None):
    """Differentiable batched sweep: returns flat (positions, normals); use
    batch.view(flat, k) for sweep k's (3, n_u, n_v) block.  path_ctrl and
    prof_ctrl are the packed (sum n, 3) float64 device tensors."""
    return SweepFunction.apply(path_ctrl, prof_ctrl, batch, out_dtype, initial_normal)
