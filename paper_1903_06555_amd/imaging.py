"""Imaging with the measurement operator: power-method normalisation and
sparse solvers.

The paper normalises Phi by its largest singular value (found with the power
method) and solves the constrained sparsity problem of Eq. (10),

    min_x ||Psi^dagger x||_1   subject to  ||y - Phi x||_2 <= eps,

with ADMM.  Here the sky is sparse in the pixel basis (point sources), so
Psi = I, and x >= 0 is added.  ``admm_l1_ball`` solves that problem by ADMM
on the split r = Phi x - y (r projected on the eps-ball, x by one
forward-backward step per iteration, the linearised ADMM of the constrained
form); ``fista_l1`` (Beck & Teboulle 2009) solves the penalised form

    min_x  1/2 ||Phi x - y||^2 + lam ||x||_1   subject to  x >= 0.

Each iteration of either costs one degrid and one grid; the proximal steps
(soft threshold and projection on x >= 0), the ball projection and the
momentum are elementwise.

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


@dataclasses.dataclass
class AdmmResult:
    x: torch.Tensor
    residual: list      # ||Phi x - y|| after every iteration
    l1: list            # ||x||_1 after every iteration
    iterations: int
    step: float


def _norm(v: torch.Tensor) -> float:
    return float(torch.sqrt(torch.sum(v.real.double() ** 2 + v.imag.double() ** 2)))


def admm_l1_ball(op, y: torch.Tensor, eps: float, mu: float, n_iter: int = 200,
                 norm2: float | None = None, x0: torch.Tensor | None = None) -> AdmmResult:
    """ADMM for min ||x||_1 subject to ||Phi x - y|| <= eps and x >= 0 (Eq. (10), Psi = I).

    Split r = Phi x - y with r in the eps-ball; scaled dual z.  Per iteration:
        r <- P_ball(Phi x - y + z)
        x <- max(x - tau Re Phi^dagger (Phi x - y - r + z) - tau mu, 0)
        z <- z + Phi x - y - r
    with tau = 1 / (1.02 ||Phi||^2) (the linearised x-step converges for
    tau ||Phi||^2 <= 1; the power method's estimate is a lower bound) and mu
    the weight of the l1 term against the augmented penalty.
    """
    L = norm2 if norm2 is not None else power_norm2(op)
    tau = 1.0 / (1.02 * L)
    x = torch.zeros(op.n, op.n, device=op.device, dtype=op.real_dtype) if x0 is None else x0.clone()
    p = op.degrid(x)
    z = torch.zeros_like(y)
    res, l1 = [], []
    for _ in range(n_iter):
        v = p - y + z
        nv = _norm(v)
        r = v if nv <= eps else v * (eps / nv)
        g = op.grid(p - y - r + z)
        x = torch.clamp(x - tau * g - tau * mu, min=0.0)
        p = op.degrid(x)
        z = z + p - y - r
        res.append(_norm(p - y))
        l1.append(float(torch.sum(torch.abs(x.double()))))
    return AdmmResult(x=x, residual=res, l1=l1, iterations=n_iter, step=tau)
