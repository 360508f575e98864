"""Differentiable matching-based OT loss (torch.autograd.Function).

Forward: the batched push-relabel solve on the HIP library gives each
instance's matching, then the library's loss kernel returns
L_i = (1/n) sum_b ||x_b - y_mate(b)||^2. Backward: the library's gradient
kernel for the fixed matching. This module only marshals tensors."""
from __future__ import annotations

import torch

from ._lib import context


class OTMatchLoss(torch.autograd.Function):
    """X, Y: (batch, n, d) float32 CUDA tensors; returns a (batch,) loss."""

    @staticmethod
    def forward(ctx, X, Y, eps: float, eps_mode: str = "algorithmic"):
        if X.dim() != 3 or Y.shape != X.shape:
            raise ValueError("X and Y must have the same (batch, n, d) shape")
        batch, n, d = X.shape
        Xp = X.detach().contiguous().view(batch * n, d)
        Yp = Y.detach().contiguous().view(batch * n, d)
        plan = context(X.device.index).cached_batch([n] * batch, d, eps, eps_mode=eps_mode)
        plan.run(Xp, Yp)
        loss = plan.loss(Xp, Yp)
        ctx.plan = plan
        ctx.shape = (batch, n, d)
        ctx.save_for_backward(Xp, Yp, plan.mate_a.clone(), plan.mate_b.clone())
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        Xp, Yp, mate_a, mate_b = ctx.saved_tensors
        dX, dY = ctx.plan.loss_grad(Xp, Yp, grad_loss, mate_a, mate_b)
        return dX.view(ctx.shape), dY.view(ctx.shape), None, None


def ot_match_loss(X, Y, eps: float, eps_mode: str = "algorithmic"):
    return OTMatchLoss.apply(X, Y, eps, eps_mode)
