"""Differentiable amplitude loss: a torch.autograd.Function whose forward
and backward both run in libptyc's kernels.  The forward runs the row and
column FFTs of P * S_j O, the loss and the hand-written adjoint
(accumulating dL/dO over overlapping windows and dL/dP in a fixed order) in
one enqueued pass, without waiting for the GPU; the backward scales the
saved gradients by the upstream gradient."""
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
        # loss and, when an input needs it, both gradients in one pass of
        # the kernels; nothing here waits for the GPU
        grad = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
        loss, flat, g_obj, g_probe = engine._amp_loss_flat(obj, probe, idx, grad)
        ctx.engine = engine
        ctx.grads = (flat, g_obj, g_probe)
        return loss

    @staticmethod
    def backward(ctx, grad_out):
        flat, g_obj, g_probe = ctx.grads
        ctx.grads = None
        # the upstream gradient scales the saved gradients, both in one
        # library call (they share one buffer)
        ctx.engine.scale_(flat, grad_out)
        return g_obj, g_probe, None, None


def amplitude_loss(engine, obj, probe, idx):
    """Functional form of AmplitudeLoss."""
    return AmplitudeLoss.apply(obj, probe, engine, idx)
