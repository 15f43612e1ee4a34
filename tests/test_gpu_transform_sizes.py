"""GPU parity of the transforms F and F^dagger (Eqs. (4), (7)) at every grid size
they are built for, on both precisions, through the whole operator.

The LDS-resident transforms run for G = 2^m up to 8192 with N <= G / 2; their
pass structure depends on G (radix-16 passes, then one of radix 2, 4 or 8, or
none).  Grids of 64, 256, 512 and 1024 cells take the tails radix 4, none, 2
and 4 (128, 2048, 4096 and 8192 are covered by the other operator tests);
N = 80 on 256 cells leaves ragged 64 x 64 transpose tiles and N < G / 2;
192 cells (a multiple of 64 that is not a power of two), and 64 cells with
N = G, take the library passes.  Every visibility and every pixel is
compared with the FP64 oracle, element by element against the largest
output: FP64 path <= 1e-7, FP32 path <= 1e-5.  The FP64 bar is set by the
kernel taps, not the transforms (an indexing error would be of order one):
their quadrature tolerance is 1e-6 of the peak, and they land within a few
1e-9 at oversampling 2 and about 4e-8 at 3.2, where the integral of
Eq. (6) runs to r = 1.6.  Three w-stacks with folding, so that the
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
CASES = [(32, 2.0, 1), (128, 2.0, 1), (256, 2.0, 1), (512, 2.0, 1), (80, 3.2, 1), (96, 2.0, 0), (64, 1.0, 0)]


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
    # the taps' own accuracy (the bar of the operator comparison below)
    tap_err = 0.0
    for p in range(0, ref.m, 10):
        K, u0, v0 = op.kernel(p)
        ru0, rv0, Kr = ref.kernel(p)
        assert (u0, v0) == (ru0, rv0)
        tap_err = max(tap_err, float(np.max(np.abs(K - Kr)) / np.max(np.abs(Kr))))
    assert tap_err <= 1e-6
    x = syn.point_source_sky(n, 12, "exp", seed=n + 1)
    y = op.degrid(torch.from_numpy(x)).cpu().numpy()
    ey = max_rel(y, ref.forward(x))
    yin = syn.random_vis(ref.m, seed=n + 2)
    xa = op.grid(torch.from_numpy(yin)).cpu().numpy()
    ex = max_rel(xa, ref.adjoint(yin))
    print(f"n {n} alpha {alpha} {precision} lds {lds} rows {st['fft_rows']}: taps {tap_err:.2e} "
          f"degrid {ey:.2e} grid {ex:.2e}")
    tol = 1e-7 if precision == "fp64" else 1e-5
    assert ey <= tol and ex <= tol
    op.close()
