"""Differentiable measurement operator.

``WStackDegrid.apply(x, op)`` returns y = Phi x (the HIP degridder); its
backward pass is the hand-written gridding kernel, Re Phi^dagger g.  With
PyTorch's conjugate-Wirtinger convention this is the gradient of any real
loss L(y) with respect to the real image x: for L = 1/2 ||Phi x - d||^2 the
incoming g is Phi x - d and x.grad = Re Phi^dagger (Phi x - d).
"""
from __future__ import annotations

import torch

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


def power_norm2(op: Operator, n_iter: int = 30, seed: int = 0) -> float:
    """||Phi||^2 (largest eigenvalue of Re Phi^dagger Phi) by the power method."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn(op.n, op.n, generator=g, dtype=torch.float64).to(op.device, op.real_dtype)
    x /= torch.linalg.vector_norm(x)
    lam = 0.0
    for _ in range(n_iter):
        z = op.grid(op.degrid(x))
        lam = float(torch.sum(z.double() * x.double()))
        x = z / torch.linalg.vector_norm(z)
    return lam
