"""Adjoint identity of an operator pair at full size (test infrastructure)."""
import numpy as np
import torch

from paper_1903_06555_amd import synthetic as syn

def adjoint_gap(op, x_np, seed):
    """|<Phi x, y> - <x, Phi^dagger y>| / |<Phi x, y>| for y = Phi x + r, r random
    of the same rms: the inner product is then ~||Phi x||^2 rather than a sum of
    random signs ~sqrt(M) times smaller than its terms, so the relative gap
    measures the operator pair's arithmetic, not cancellation."""
    xr = torch.from_numpy(x_np)
    Phx = op.degrid(xr).cpu().numpy().astype(np.complex128)
    r = syn.random_vis(Phx.size, seed=seed)
    y = Phx + r * (np.linalg.norm(Phx) / np.linalg.norm(r))
    Phty = op.grid(torch.from_numpy(y)).cpu().numpy().astype(np.float64)
    lhs = float(np.real(np.vdot(Phx, y)))
    rhs = float(np.sum(x_np * Phty))
    return abs(lhs - rhs) / abs(lhs)
