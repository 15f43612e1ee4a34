"""Pins of the oracle's DDE convolution (Eq. (11)), CPU only.

Facts that hold independently of the convolution code:
- a centred delta D leaves the kernel unchanged (padded by h zeros);
- the convolution theorem: the zero-padded 2-D DFT of D * K is the product
  of those of D and K;
- Fourier shift theorem: D = a unit delta one cell to +u moves every tap one
  cell to +u, so the operator equals the plain operator at u + du (any
  transposition or flip of the convolution breaks this);
- the operator with D stays self-consistent (adjoint identity).
"""
import math

import numpy as np

from oracle import dde, operator, wkernel
from paper_1903_06555_amd import synthetic as syn

GEOM = wkernel.Geometry(n=32, fov=math.radians(10.0))


def random_dde(m, jd, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(m, jd)) + 1j * rng.normal(size=(m, jd)),
            rng.normal(size=(m, jd)) + 1j * rng.normal(size=(m, jd)))


def test_delta_leaves_kernel():
    u0, v0, K = wkernel.visibility_kernel(3.3, -2.7, 11.0, GEOM)
    d = np.zeros(5, dtype=complex)
    d[2] = 1.0
    Kc = dde.convolve_kernel(K, d, d)
    jp = K.shape[0]
    assert Kc.shape == (jp + 4, jp + 4)
    assert np.array_equal(Kc[2:-2, 2:-2], K)
    assert not np.any(Kc[:2]) and not np.any(Kc[-2:]) and not np.any(Kc[:, :2]) and not np.any(Kc[:, -2:])


def test_convolution_theorem():
    _, _, K = wkernel.visibility_kernel(0.4, 0.9, 23.0, GEOM)
    du, dv = random_dde(1, 7, 81)
    Kc = dde.convolve_kernel(K, du[0], dv[0])
    S = Kc.shape
    D = np.outer(dv[0], du[0])
    lhs = np.fft.fft2(Kc, s=S)
    rhs = np.fft.fft2(K, s=S) * np.fft.fft2(D, s=S)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs))


def test_unit_shift_is_the_operator_at_shifted_u():
    uvw = syn.uniform_box_uvw(300, u_max=25.0, w_max=15.0, seed=82)
    plain = operator.StackedOperator(GEOM, uvw, n_stacks=2)
    m = plain.m
    du = np.zeros((m, 3), dtype=complex)
    dv = np.zeros((m, 3), dtype=complex)
    du[:, 2] = 1.0   # offset +1 cell in u
    dv[:, 1] = 1.0   # no shift in v
    shifted_op = operator.StackedOperator(GEOM, uvw, labels=plain.labels, centres=plain.centres,
                                          kernel_fn=dde.DDEKernels(du, dv), extra_support=2)
    uvw_s = uvw.copy()
    uvw_s[:, 0] += GEOM.du
    ref = operator.StackedOperator(GEOM, uvw_s, labels=plain.labels, centres=plain.centres)
    x = syn.point_source_sky(32, 5, "gaussian", seed=83, margin=3)
    y, y_ref = shifted_op.forward(x), ref.forward(x)
    assert np.max(np.abs(y - y_ref)) <= 1e-12 * np.max(np.abs(y_ref))
    # and it is not the unshifted operator
    assert np.linalg.norm(y - plain.forward(x)) > 1e-3 * np.linalg.norm(y)


def test_adjoint_identity_with_dde():
    uvw = syn.uniform_box_uvw(200, u_max=25.0, w_max=15.0, seed=84)
    du, dv = random_dde(200, 5, 85)
    op = operator.StackedOperator(GEOM, uvw, n_stacks=2, fold=True,
                                  kernel_fn=dde.DDEKernels(du, dv), extra_support=4)
    assert np.array_equal(op.jp, dde.support(op.w_eff, GEOM, 5))
    x = syn.point_source_sky(32, 5, "gaussian", seed=86, margin=3)
    yr = syn.random_vis(op.m, seed=87)
    lhs = float(np.real(np.vdot(op.forward(x), yr)))
    rhs = float(np.sum(x * op.adjoint(yr)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
