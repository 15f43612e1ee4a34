"""Pins of the oracle's w-plane interpolation (Sec. 5.1.1), CPU only.

Checks that do not rely on the interpolation code being right:
- a lattice filled from a bilinear function f = a + b q + c w + d q w is
  reproduced exactly (a swapped weight, a wrong index or a transposed lattice
  breaks it);
- at lattice nodes the interpolant is the quadrature value;
- K~(q, -w) = conj K~(q, w), and it is close to the direct kernel at -w
  (Sec. 5.1.1: conjugation covers negative w);
- the error against the direct Eq. (6) kernel is within the textbook bound of
  bilinear interpolation, h_q^2/8 max|d2K/dq2| + h_w^2/8 max|d2K/dw2|, with
  the second derivatives measured on the direct kernel, and falls about
  fourfold when both steps are halved;
- the operator built from interpolated kernels agrees with the exact-kernel
  operator to the interpolation level, far below the aliasing level.
"""
import math

import numpy as np
import pytest

from oracle import operator, presample, wkernel
from paper_1903_06555_amd import synthetic as syn

GEOM = wkernel.Geometry(n=1024, fov=math.radians(25.0))


def test_bilinear_reproduces_bilinear_functions():
    rng = np.random.default_rng(7)
    a, b, c, d = rng.normal(size=4) + 1j * rng.normal(size=4)
    dq, dw = 0.05, 0.3

    def lattice(j, idx):
        return a + b * (np.asarray(idx) * dq) + c * (j * dw) + d * (np.asarray(idx) * dq) * (j * dw)

    q = rng.uniform(0.0, 20.0, 500)
    for w in rng.uniform(0.0, 40.0, 20):
        exact = a + b * q + c * w + d * q * w
        got = presample.bilinear(lattice, q, w, dq, dw)
        assert np.max(np.abs(got - exact)) <= 1e-12 * np.max(np.abs(exact))
        neg = presample.bilinear(lattice, q, -w, dq, dw)
        assert np.array_equal(neg, np.conj(got))


def test_nodes_equal_quadrature():
    ps = presample.PlaneSampler(GEOM)
    i = np.arange(0, 900, 7)
    for j in (0, 3, 161):
        direct = wkernel.wkernel(i * ps.dq, j * ps.dw, GEOM)
        assert np.max(np.abs(ps.kernel(i * ps.dq, j * ps.dw) - direct)) <= 1e-13 * np.max(np.abs(direct))


def second_derivative_bounds(w0, qmax, dq, dw):
    """max |d2K/dq2| and max |d2K/dw2| near (q in [0, qmax], w ~ w0), by central differences."""
    hq = 1.0 / 256.0
    q = np.arange(0.0, qmax + dq, hq / 2)
    K = wkernel.wkernel(q, w0, GEOM)
    kqq = np.max(np.abs(K[2:] - 2 * K[1:-1] + K[:-2])) / (hq / 2) ** 2
    hw = dw / 4
    kww = 0.0
    for wc in (w0, w0 + dw / 2, w0 + dw):
        Km, K0, Kp = (wkernel.wkernel(q[::8], wc + e, GEOM) for e in (-hw, 0.0, hw))
        kww = max(kww, float(np.max(np.abs(Kp - 2 * K0 + Km))) / hw ** 2)
    return kqq, kww


@pytest.mark.parametrize("w", [0.02, 12.3, 151.7])
def test_error_within_bilinear_bound(w):
    dq, dw = presample.DEFAULT_DQ, presample.DEFAULT_DW
    jp = int(wkernel.support(w, GEOM))
    qmax = jp / math.sqrt(2.0)
    rng = np.random.default_rng(11)
    q = rng.uniform(0.0, qmax, 150)
    # w values in the same lattice cell as w, so the w-curvature is measured there
    ws = math.floor(w / dw) * dw + rng.uniform(0.0, dw, 3)
    kqq, kww = second_derivative_bounds(math.floor(w / dw) * dw, qmax, dq, dw)
    bound = 1.5 * (dq * dq / 8.0 * kqq + dw * dw / 8.0 * kww)  # 1.5: sampled maxima
    ps = presample.PlaneSampler(GEOM, dq, dw)
    err = 0.0
    for wv in ws:
        err = max(err, float(np.max(np.abs(ps.kernel(q, wv) - wkernel.wkernel(q, wv, GEOM)))))
    peak = float(np.max(np.abs(wkernel.wkernel(np.linspace(0, 2, 9), w, GEOM))))
    assert err <= bound, (err, bound)
    assert err <= 2e-4 * peak, err / peak  # the default steps' design level
    # halving both steps: about four times smaller
    ps2 = presample.PlaneSampler(GEOM, dq / 2, dw / 2)
    err2 = max(float(np.max(np.abs(ps2.kernel(q, wv) - wkernel.wkernel(q, wv, GEOM)))) for wv in ws)
    assert err2 <= err / 2.5, (err, err2)


def test_negative_w_is_conjugate():
    ps = presample.PlaneSampler(GEOM)
    q = np.linspace(0.0, 10.0, 97)
    for w in (3.3, 40.01):
        kp, kn = ps.kernel(q, w), ps.kernel(q, -w)
        assert np.array_equal(kn, np.conj(kp))
        direct = wkernel.wkernel(q, -w, GEOM)
        assert np.max(np.abs(kn - direct)) <= 2e-4 * np.max(np.abs(direct))


def test_operator_with_plane_kernels_matches_exact_operator():
    # 64^2 image, 25 deg, visibilities with |w| <= 30 (supports up to 22 taps)
    geom = wkernel.Geometry(n=64, fov=math.radians(25.0))
    uvw = syn.uniform_box_uvw(300, u_max=60.0, w_max=30.0, seed=31)
    ps = presample.PlaneSampler(geom)
    exact = operator.StackedOperator(geom, uvw, n_stacks=2, fold=True)
    planes = operator.StackedOperator(geom, uvw, labels=exact.labels, centres=exact.centres,
                                      fold=True, kernel_fn=ps.visibility_kernel)
    x = syn.point_source_sky(64, 8, "exp", seed=32, margin=4)
    ye, yp = exact.forward(x), planes.forward(x)
    rel = float(np.linalg.norm(yp - ye) / np.linalg.norm(ye))
    assert 0.0 < rel <= 2e-4, rel
    # the plane operator's adjoint is its adjoint
    yr = syn.random_vis(exact.m, seed=33)
    lhs = float(np.real(np.vdot(planes.forward(x), yr)))
    rhs = float(np.sum(x * planes.adjoint(yr)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
