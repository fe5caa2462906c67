"""Differentiable slicing: the backward of the type-2 NUFFT is its type-1
adjoint (the merging operator A* of section II-C, Eq. (2)), run by the
library's spread kernels.

* ``SliceFn``: slices = A(model); grad_model = A^H grad_slices.
* ``SliceLossFn``: L = sum_{n,p} w_np |A_n(model)_p - d_np|^2 computed in
  chunks of images without keeping the slices; the backward recomputes each
  chunk's slices and spreads 2 w (s - d): grad = 2 A^H (W (A m - d)).
"""
from __future__ import annotations

import torch

from . import ops


class SliceFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, quats, det_q, plan):
        plan.set_model(model.contiguous())
        s, _ = plan.slice(quats, det_q)
        ctx.save_for_backward(quats, det_q)
        ctx.plan = plan
        return s

    @staticmethod
    def backward(ctx, grad_s):
        quats, det_q = ctx.saved_tensors
        g = ctx.plan.merge_adjoint(quats, det_q, grad_s.contiguous())
        return g, None, None, None


def slice_model(model, quats, det_q, plan):
    return SliceFn.apply(model, quats, det_q, plan)


class SliceLossFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model, quats, det_q, images, weights, plan, chunk):
        plan.set_model(model.contiguous())
        loss = torch.zeros((), dtype=torch.float64, device=model.device)
        n = quats.shape[0]
        for c0 in range(0, n, chunk):
            c1 = min(n, c0 + chunk)
            s, _ = plan.slice(quats[c0:c1], det_q)
            w = None if weights is None else weights[c0:c1]
            plan.weighted_residual(s, images[c0:c1], w, residual=False, loss=loss)
            del s
        ctx.save_for_backward(model, quats, det_q, images, weights)
        ctx.plan = plan
        ctx.chunk = chunk
        return loss.to(torch.float32)

    @staticmethod
    def backward(ctx, grad_loss):
        model, quats, det_q, images, weights = ctx.saved_tensors
        plan, chunk = ctx.plan, ctx.chunk
        # the incoming factor stays on the device (no host round trip)
        g_dev = grad_loss.detach().to(torch.float32).reshape(1).contiguous()
        plan.set_model(model.contiguous())
        n = quats.shape[0]
        grad = None
        for c0 in range(0, n, chunk):
            c1 = min(n, c0 + chunk)
            s, _ = plan.slice(quats[c0:c1], det_q)
            w = None if weights is None else weights[c0:c1]
            r, _ = plan.weighted_residual(s, images[c0:c1], w, scale=2.0, residual=True,
                                          scale_dev=g_dev)
            del s
            last = c1 == n
            grad = plan.merge_adjoint(quats[c0:c1], det_q, r,
                                      flags=0 if last else ops.MERGE_DEFER)
        return grad, None, None, None, None, None, None


def slice_loss(model, quats, det_q, images, weights, plan, chunk: int = 1024):
    return SliceLossFn.apply(model, quats, det_q, images, weights, plan, chunk)
