"""Imaging with the measurement operator: power-method normalisation and a
sparse least-squares solver.

The paper normalises Phi by its largest singular value (found with the power
method) and solves a sparsity-regularised problem with ADMM (Sec. 3, Eq. 10).
Here the sky is sparse in the pixel basis (point sources), and the solver is
FISTA (Beck & Teboulle 2009) for

    min_x  1/2 ||Phi x - y||^2 + lam ||x||_1   subject to  x >= 0,

whose gradient step is one degrid and one grid; the proximal step (soft
threshold and projection on x >= 0) and the momentum are elementwise.

The functions take any operator object with ``degrid(x)``, ``grid(y)``,
``n``, ``device`` and ``real_dtype`` (``wsp.Operator`` on the GPU).
"""
from __future__ import annotations

import dataclasses
import math

import torch


def power_norm2(op, n_iter: int = 50, tol: float = 1e-9, seed: int = 0) -> float:
    """||Phi||^2, the largest eigenvalue of Re Phi^dagger Phi, by power iteration.

    Returns the Rayleigh quotient, which approaches ||Phi||^2 from below (slowly
    when the two largest eigenvalues are close); stops when it changes by less
    than ``tol`` (relative).
    """
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn(op.n, op.n, generator=g, dtype=torch.float64).to(op.device, op.real_dtype)
    x = x / torch.linalg.vector_norm(x)
    lam = 0.0
    for _ in range(n_iter):
        z = op.grid(op.degrid(x))
        new = float(torch.sum(z.double() * x.double()))
        x = z / torch.linalg.vector_norm(z)
        if lam and abs(new - lam) <= tol * abs(new):
            lam = new
            break
        lam = new
    return lam


@dataclasses.dataclass
class FistaResult:
    x: torch.Tensor
    objective: list
    iterations: int
    step: float


def objective(op, x: torch.Tensor, y: torch.Tensor, lam: float) -> float:
    r = op.degrid(x) - y
    return 0.5 * float(torch.sum(r.real.double() ** 2 + r.imag.double() ** 2)) + \
        lam * float(torch.sum(torch.abs(x.double())))


def fista_l1(op, y: torch.Tensor, lam: float, n_iter: int = 100, norm2: float | None = None,
             x0: torch.Tensor | None = None, track: bool = True) -> FistaResult:
    """FISTA for 1/2 ||Phi x - y||^2 + lam ||x||_1 with x >= 0.

    ``norm2`` is ||Phi||^2 (the Lipschitz constant of the gradient); computed
    with the power method if not given.  The step is 1 / (1.02 norm2): the
    power method's estimate is a lower bound, and FISTA converges only for
    steps up to 1 / ||Phi||^2.  With ``track`` the objective is evaluated
    after every iteration (one extra degrid each).
    """
    L = norm2 if norm2 is not None else power_norm2(op)
    step = 1.0 / (1.02 * L)
    x = torch.zeros(op.n, op.n, device=op.device, dtype=op.real_dtype) if x0 is None else x0.clone()
    z = x.clone()
    t = 1.0
    hist = []
    for _ in range(n_iter):
        grad = op.grid(op.degrid(z) - y)  # Re Phi^dagger (Phi z - y)
        x_new = torch.clamp(z - step * grad - step * lam, min=0.0)
        t_new = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
        z = x_new + ((t - 1.0) / t_new) * (x_new - x)
        x, t = x_new, t_new
        if track:
            hist.append(objective(op, x, y, lam))
    return FistaResult(x=x, objective=hist, iterations=n_iter, step=step)
