"""Differentiable amplitude loss: a torch.autograd.Function whose forward
and backward both run in libptyc's kernels (forward: row and column FFTs of
P * S_j O and the loss; backward: the hand-written adjoint, accumulating
dL/dO over overlapping windows and dL/dP in a fixed order)."""
from __future__ import annotations

import torch


class AmplitudeLoss(torch.autograd.Function):
    """L(O, P) = sum_{j in idx} sum_k (|F(P * S_j O)|_k - sqrt(I_j,k))^2.

    ``engine`` holds the measured patterns and scan positions; ``obj``
    (H x W) and ``probe`` (N x N) are complex64 CUDA tensors.  Gradients
    follow PyTorch's convention (dL/dRe + i dL/dIm), so torch.optim works on
    the complex parameters directly."""

    @staticmethod
    def forward(ctx, obj, probe, engine, idx):
        loss = engine.amp_loss(obj, probe, idx)
        ctx.engine = engine
        ctx.idx = idx
        ctx.save_for_backward(obj, probe)
        return torch.tensor(loss, dtype=torch.float64, device=obj.device)

    @staticmethod
    def backward(ctx, grad_out):
        obj, probe = ctx.saved_tensors
        scale = float(grad_out)
        _, g_obj, g_probe = ctx.engine.amp_loss(obj, probe, ctx.idx, grad=True, scale=scale)
        return g_obj, g_probe, None, None


def amplitude_loss(engine, obj, probe, idx):
    """Functional form of AmplitudeLoss."""
    return AmplitudeLoss.apply(obj, probe, engine, idx)
