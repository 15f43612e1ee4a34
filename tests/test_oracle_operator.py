"""Pins for oracle.operator (Eqs. (2)-(8)) against the direct DFT and identities."""
import math

import numpy as np
import pytest

from oracle import dft, operator, wkernel
from paper_1903_06555_amd import synthetic as syn

GEOM = wkernel.Geometry(n=64, fov=math.radians(10.0))


@pytest.fixture(scope="module")
def tiny():
    wl = syn.WORKLOADS["tiny_box_64"]
    return syn.workload_uvw(wl), syn.workload_sky(wl)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_forward_matches_direct_dft_at_aliasing_level(tiny):
    uvw, x = tiny
    y = operator.StackedOperator(GEOM, uvw).forward(x)
    yd = dft.measure(x, uvw, GEOM.fov)
    uvw0 = uvw.copy()
    uvw0[:, 2] = 0.0
    e0 = _rel(operator.StackedOperator(GEOM, uvw0).forward(x), dft.measure(x, uvw0, GEOM.fov))
    e = _rel(y, yd)
    assert e < 1e-2 and e < 3 * e0, (e, e0)


def test_w0_radial_and_separable_kb_agree_with_dft_at_same_level(tiny):
    uvw, x = tiny
    uvw0 = uvw.copy()
    uvw0[:, 2] = 0.0
    yd = dft.measure(x, uvw0, GEOM.fov)
    e_rad = _rel(operator.StackedOperator(GEOM, uvw0).forward(x), yd)
    e_sep = _rel(operator.separable_kb_forward(GEOM, x, uvw0), yd)
    assert e_rad < 1e-2 and e_sep < 1e-2
    assert e_rad < 3 * e_sep and e_sep < 3 * e_rad


def test_adjoint_dot_product_with_fold_weights_and_stacks():
    uvw = syn.uniform_box_uvw(300, seed=11)
    wts = syn.random_weights(300, seed=12)
    op = operator.StackedOperator(GEOM, uvw, weights=wts, n_stacks=3, fold=True)
    x = syn.random_image(GEOM.n, seed=13)
    y = syn.random_vis(300, seed=14)
    lhs = np.real(np.vdot(op.forward(x), y))
    rhs = np.sum(x * op.adjoint(y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_stack_count_does_not_change_the_model(tiny):
    # Eq. (7): stacking only moves w between S~_k and GC_k
    uvw, x = tiny
    yd = dft.measure(x, uvw, GEOM.fov)
    y1 = operator.StackedOperator(GEOM, uvw, n_stacks=1).forward(x)
    y4 = operator.StackedOperator(GEOM, uvw, n_stacks=4).forward(x)
    assert _rel(y4, yd) < 1e-2
    assert _rel(y4, y1) < 1e-2


def test_fold_identity_is_exact(tiny):
    uvw, x = tiny
    neg = uvw[:, 2] < 0
    flipped = uvw.copy()
    flipped[neg] = -flipped[neg]
    opf = operator.StackedOperator(GEOM, uvw, fold=True, n_stacks=2)
    opn = operator.StackedOperator(GEOM, flipped, fold=False, labels=opf.labels, centres=opf.centres)
    yf = opf.forward(x)
    yn = opn.forward(x)
    assert np.array_equal(yf[neg], np.conj(yn[neg]))
    assert np.array_equal(yf[~neg], yn[~neg])
    assert _rel(yf, dft.measure(x, uvw, GEOM.fov)) < 1e-2


def test_wide_field_large_w_converges_to_dft_as_support_grows():
    # 25 deg, |w| up to ~20: the corner-bandwidth support leaves a truncation
    # error of a few 1e-2; widening the support drives it to the w = 0 level.
    uvw = syn.mwa_rotation_uvw(8128, 120.0)[::40][:120] * 0.04
    x = syn.point_source_sky(128, 30, "exp", seed=2, margin=8)
    errs = []
    for f in [1.0, 2.0, 4.0]:
        geom = wkernel.Geometry(n=128, fov=math.radians(25.0), support_scale=f)
        op = operator.StackedOperator(geom, uvw, n_stacks=1)
        errs.append(_rel(op.forward(x), dft.measure(x, uvw, geom.fov)))
    geom = wkernel.Geometry(n=128, fov=math.radians(25.0))
    uvw0 = uvw.copy()
    uvw0[:, 2] = 0.0
    e0 = _rel(operator.StackedOperator(geom, uvw0).forward(x), dft.measure(x, uvw0, geom.fov))
    assert errs[0] < 5e-2
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 3 * e0, (errs, e0)


def test_forward_at_and_adjoint_at_equal_the_fft_route():
    """The cell-wise DFT evaluation equals the numpy FFT route, element by
    element, with stacks, fold and weights, for sparse and dense images."""
    uvw = syn.uniform_box_uvw(400, u_max=55.0, w_max=30.0, seed=31)
    wts = syn.random_weights(400, seed=32)
    op = operator.StackedOperator(GEOM, uvw, weights=wts, n_stacks=3, fold=True)
    subset = np.random.default_rng(33).permutation(400)[:90]   # unsorted on purpose
    for x in (syn.point_source_sky(GEOM.n, 25, "exp", 34), syn.random_image(GEOM.n, 35)):
        y_fft = op.forward(x, subset=subset)
        y_at = op.forward_at(x, subset)
        assert np.count_nonzero(y_at) == subset.size
        assert np.max(np.abs(y_at - y_fft)) <= 1e-12 * np.max(np.abs(y_fft))
    y = np.zeros(400, dtype=np.complex128)
    y[subset] = syn.random_vis(subset.size, seed=36)
    x_fft = op.adjoint(y, subset=subset)
    rng = np.random.default_rng(37)
    rows = np.concatenate([[0, GEOM.n - 1, GEOM.n // 2], rng.integers(0, GEOM.n, 200)])
    cols = np.concatenate([[0, GEOM.n - 1, GEOM.n // 2], rng.integers(0, GEOM.n, 200)])
    x_at = op.adjoint_at(y, rows, cols, subset)
    assert np.max(np.abs(x_at - x_fft[rows, cols])) <= 1e-12 * np.max(np.abs(x_fft))
