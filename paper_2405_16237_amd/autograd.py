"""Differentiable N-BVH network outputs for PyTorch.

NBVHFunction.apply(params, probes, model) returns z = f(probes; params) for
probe segments through the library's fused forward kernel; its backward calls
the library's back-propagation (encodings and activations are recomputed, not
stored) and returns dL/dparams in the library's padded parameter layout.
`params` must be `model.params` (the buffer the library reads); a torch
optimiser may update it in place between calls.
"""
from __future__ import annotations

import torch

from .nbvh import NBVH


class NBVHFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params: torch.Tensor, probes: torch.Tensor, model: NBVH):
        if params.data_ptr() != model.params.data_ptr():
            raise ValueError("params must be model.params (the buffer bound to the library)")
        if model.precision != 0:
            model.sync_shadow()  # params may have been edited since the last optimiser step
        z = model.forward(probes)
        ctx.model = model
        ctx.save_for_backward(probes)
        return z

    @staticmethod
    def backward(ctx, dz: torch.Tensor):
        model = ctx.model
        (probes,) = ctx.saved_tensors
        model.grad.zero_()
        model.backward(probes, dz.contiguous().float())
        # the library divides out its loss scale and clears its accumulator
        g = model.unscaled_grad(clear=True)
        return g, None, None


def nbvh_forward(model: NBVH, probes: torch.Tensor) -> torch.Tensor:
    """z for probe segments, differentiable with respect to model.params."""
    if not model.params.requires_grad:
        model.params.requires_grad_(True)
    return NBVHFunction.apply(model.params, probes, model)
