"""wsp_build_kernels_noalloc against wsp_build_kernels, through the C ABI.

The no-alloc build runs the same kernels on batches carved from a static
device workspace, so its taps must equal the allocating build's bit for bit.
Two calls in a row, the second on a smaller problem (the workspace keeps the
first call's contents); the kernel buffer is poisoned before each no-alloc
build so that every tap must be written by it.
"""
import math

import numpy as np
import pytest
import torch

from paper_1903_06555_amd import synthetic as syn
from paper_1903_06555_amd import wsp

pytestmark = pytest.mark.gpu

CASES = [
    # (n, M, stacks, fold, precision): the first needs several static batches
    (512, 30_000, 1, False, "fp32_fp64phase"),
    (256, 5_000, 4, True, "fp64"),
]


def _check_case(n, m, stacks, fold, precision):
    uvw = syn.mwa_rotation_uvw(m, 600.0)
    params = wsp.make_params(n, math.radians(25.0), n_stacks=stacks, fold=fold, precision=precision)
    op = wsp.Operator(params, uvw, build=False)
    kb = op.footprint["kernel_bytes"]
    assert wsp.wsp_build_kernels(op.ctx) == wsp.WSP_OK
    torch.cuda.synchronize()
    ref = op.kernels[:kb].clone()
    ref_stats = op.quad_stats()
    op.kernels.fill_(255)  # NaN bytes: a tap the no-alloc build skipped would show
    torch.cuda.synchronize()
    assert wsp.wsp_build_kernels_noalloc(op.ctx) == wsp.WSP_OK
    torch.cuda.synchronize()
    got = op.kernels[:kb]
    same = bool(torch.equal(got, ref))
    n_diff = int((got != ref).sum()) if not same else 0
    print(f"n={n} M={m} K={stacks} {precision}: {kb} kernel bytes, differing bytes {n_diff}", flush=True)
    assert same
    assert op.quad_stats() == ref_stats
    # the operator runs on the no-alloc build
    x = torch.from_numpy(syn.point_source_sky(n, 30, "exp", 5))
    y = op.degrid(x).cpu().numpy()
    assert np.isfinite(y).all() and np.abs(y).max() > 0
    op.close()


def test_noalloc_build_equals_allocating_build_twice_second_smaller():
    assert CASES[1][1] < CASES[0][1]
    for case in CASES:
        _check_case(*case)
