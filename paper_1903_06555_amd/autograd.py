"""Differentiable measurement operator.

``WStackDegrid.apply(x, op)`` returns y = Phi x (the HIP degridder); its
backward pass is the hand-written gridding kernel, Re Phi^dagger g.  With
PyTorch's conjugate-Wirtinger convention this is the gradient of any real
loss L(y) with respect to the real image x: for L = 1/2 ||Phi x - d||^2 the
incoming g is Phi x - d and x.grad = Re Phi^dagger (Phi x - d).
"""
from __future__ import annotations

import torch

from .imaging import power_norm2  # noqa: F401  (||Phi||^2 for step sizes)
from .wsp import Operator


class WStackDegrid(torch.autograd.Function):
    @staticmethod
    def forward(ctx, image: torch.Tensor, op: Operator):
        ctx.op = op
        return op.degrid(image)

    @staticmethod
    def backward(ctx, grad_vis: torch.Tensor):
        return ctx.op.grid(grad_vis.contiguous()), None


def degrid(image: torch.Tensor, op: Operator) -> torch.Tensor:
    return WStackDegrid.apply(image, op)
