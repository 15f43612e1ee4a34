"""GPU parity of the transforms F and F^dagger (Eqs. (4), (7)) at every grid size
they are built for, on both precisions, through the whole operator.

The LDS-resident transforms run for G = 2^m up to 8192 with N <= G / 2; their
pass structure depends on G (radix-16 passes, then one of radix 2, 4 or 8, or
none).  Grids of 64, 256, 512 and 1024 cells take the tails radix 4, none, 2
and 4 (128, 2048, 4096 and 8192 are covered by the other operator tests);
192 cells (a multiple of 64 that is not a power of two), and 64 cells with
N = G, take the library passes.  Every visibility and every pixel is
compared with the FP64 oracle, element by element against the largest
output: FP64 path <= 1e-8 (the FP64 taps are within a few 1e-9 of the
kernel peak), FP32 path <= 1e-5.  Three w-stacks with folding, so that the
per-stack transforms and the stack sum are exercised.
"""
import math

import numpy as np
import pytest
import torch

from oracle import operator, wkernel
from paper_1903_06555_amd import synthetic as syn
from paper_1903_06555_amd import wsp

pytestmark = pytest.mark.gpu

FOV = math.radians(10.0)

# (n, oversample, transform path expected)
CASES = [(32, 2.0, 1), (128, 2.0, 1), (256, 2.0, 1), (512, 2.0, 1), (96, 2.0, 0), (64, 1.0, 0)]


def max_rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("precision", ["fp64", "fp32_fp64phase"])
@pytest.mark.parametrize("n,alpha,lds", CASES)
def test_transforms_every_output(n, alpha, lds, precision):
    # visibilities over most of the grid's uv extent, |w| up to 30
    u_max = 0.4 * n / FOV
    uvw = syn.uniform_box_uvw(400, u_max=u_max, w_max=30.0, seed=n)
    geom = wkernel.Geometry(n=n, fov=FOV, alpha=alpha)
    ref = operator.StackedOperator(geom, uvw, n_stacks=3, fold=True)
    params = wsp.make_params(n, FOV, oversample=alpha, n_stacks=3, fold=True, precision=precision)
    op = wsp.Operator(params, uvw, labels=ref.labels, centres=ref.centres)
    st = op.plan_stats()
    assert st["fft_lds"] == lds, (n, alpha, st["fft_lds"])
    x = syn.point_source_sky(n, 12, "exp", seed=n + 1)
    y = op.degrid(torch.from_numpy(x)).cpu().numpy()
    ey = max_rel(y, ref.forward(x))
    yin = syn.random_vis(ref.m, seed=n + 2)
    xa = op.grid(torch.from_numpy(yin)).cpu().numpy()
    ex = max_rel(xa, ref.adjoint(yin))
    print(f"n {n} alpha {alpha} {precision} lds {lds} rows {st['fft_rows']}: degrid {ey:.2e} grid {ex:.2e}")
    tol = 1e-8 if precision == "fp64" else 1e-5
    assert ey <= tol and ex <= tol
    op.close()
