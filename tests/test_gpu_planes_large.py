"""GPU parity of the w-plane kernel mode (Sec. 5.1.1) on large entries, every
output against the oracle.

With supports of 38 - 118 cells on a 256-cell grid, the work items hold
entries of up to 64 x 64 taps, so degrid and grid run their large-entry
kernels (a wavefront per entry, batches of up to 16 taps per lane, every
tap interpolated from two lattice loads).  Tiles hold more taps than one work
item takes (2^19 by default, 4096 in the second case, which cuts them into
many more items), so the split-tile reduction adds partial tiles.  The
lattice step is the default dq = 1/64 cell and 1/256, whose pair rows are
four times longer (other column indices, clamps at other row ends).

w is drawn near four values (within one plane interval of each), two of them
negative (the conjugate rule of the lattice), in one stack centred at 0.  The
oracle interpolates its FP64 lattice with the same steps
(oracle/presample.py).  Every visibility of degrid and every pixel of grid is
compared, max |dy| / max |y|: per tap the two differ by the lattice values
(quadrature tolerance, FP32 storage: a few 1e-6 of the peak) and by FP32 tap
distances (about 3e-6 q of the peak, q in cells); the sums over supports of
this size stay within 5e-5 of the largest output.
"""
import math

import numpy as np
import pytest
import torch

from oracle import operator, presample, wkernel
from paper_1903_06555_amd import synthetic as syn
from paper_1903_06555_amd import wsp

pytestmark = pytest.mark.gpu

N = 128
FOV = math.radians(25.0)
M = 300


def max_rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def problem_uvw():
    rng = np.random.default_rng(7)
    uvw = np.empty((M, 3))
    uvw[:, 0] = rng.uniform(-0.35, 0.35, M) * N / FOV
    uvw[:, 1] = rng.uniform(-0.35, 0.35, M) * N / FOV
    centres = np.array([60.0, 140.0, -90.0, -200.0])
    uvw[:, 2] = centres[rng.integers(0, 4, M)] + rng.uniform(0.0, 0.9 / 16.0, M)
    return uvw


@pytest.fixture(scope="module", params=[1.0 / 64.0, 1.0 / 256.0], ids=["dq64", "dq256"])
def case(request):
    dq = request.param
    geom = wkernel.Geometry(n=N, fov=FOV)
    uvw = problem_uvw()
    labels, centres = np.zeros(M, dtype=np.int64), np.zeros(1)
    ps = presample.PlaneSampler(geom, dq=dq)
    ref = operator.StackedOperator(geom, uvw, labels=labels, centres=centres, kernel_fn=ps.visibility_kernel)
    x = syn.point_source_sky(N, 10, "exp", seed=3, margin=4)
    yin = syn.random_vis(M, seed=4)
    return dq, uvw, labels, centres, ref, x, ref.forward(x), yin, ref.adjoint(yin)


@pytest.mark.parametrize("item_taps", [0, 4096])
def test_large_entries_every_output(case, item_taps):
    dq, uvw, labels, centres, ref, x, y_ref, yin, x_ref = case
    params = wsp.make_params(N, FOV, kernels="planes", plane_dq=dq, item_taps=item_taps)
    op = wsp.Operator(params, uvw, labels=labels, centres=centres)
    try:
        st = op.plan_stats()
        assert op.build_status == 0
        # entries large enough for the large-entry kernels
        assert st["taps"] >= 160 * st["entries"], st
        assert st["split_tiles"] > 0, st
        op.scratch.fill_(255)
        y = op.degrid(torch.from_numpy(x)).cpu().numpy()
        op.scratch.fill_(255)
        xa = op.grid(torch.from_numpy(yin)).cpu().numpy()
        ey, ex = max_rel(y, y_ref), max_rel(xa, x_ref)
        print(f"dq 1/{round(1 / dq)} item_taps {item_taps}: {st['items']} items, J_p {ref.jp.min()}-{ref.jp.max()}: "
              f"degrid {ey:.2e} grid {ex:.2e}", flush=True)
        assert ey <= 5e-5 and ex <= 5e-5
        # repeated calls are bit-identical (entries are added in a fixed order)
        op.scratch.fill_(255)
        assert np.array_equal(op.grid(torch.from_numpy(yin)).cpu().numpy(), xa)
        assert np.array_equal(op.degrid(torch.from_numpy(x)).cpu().numpy(), y)
    finally:
        op.close()
