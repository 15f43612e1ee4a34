"""Direction-dependent effects as a further convolution of the kernel (Sec. 5.2, Eq. (11)).  FP64.

Test infrastructure only.

A baseline-dependent DDE known in the uv-domain as a small discrete kernel D
(J_D x J_D grid cells, J_D odd, centred) enters the measurement operator by
convolving it with the visibility's w-projection kernel (convolution is
commutative):  GC -> D * GC.  With D separable, D[b, a] = d_v[b] d_u[a]
(a along u / columns, b along v / rows, offsets -h .. h, h = (J_D - 1) / 2):

    K'[r, c] = sum_{a, b} d_v[b] d_u[a] K[r - b, c - a],

a J_p' = J_p + J_D - 1 square support whose first tap is h cells before the
w-kernel's (U0' = U0 - h, which is U0's rule floor(u) - J_p'/2 + 1 again).
Computed here as the full 2-D convolution with the outer product D (a library
routine); the separable form (two 1-D passes, O(J^2 J_D)) is the GPU's.

Pins (tests/test_oracle_dde.py): a centred delta D returns K; the 2-D DFT of
K' equals the product of the DFTs of K and D (convolution theorem); a D that
is a one-cell shift in u turns the operator into the operator at u + du
(Fourier shift theorem, to rounding); the adjoint identity.
"""
from __future__ import annotations

import numpy as np
from scipy import signal

from . import wkernel
from .wkernel import Geometry


def convolve_kernel(K, d_u, d_v):
    """K' = D * K with D[b, a] = d_v[b] d_u[a] (full 2-D discrete convolution)."""
    D = np.outer(np.asarray(d_v, dtype=np.complex128), np.asarray(d_u, dtype=np.complex128))
    return signal.convolve2d(np.asarray(K, dtype=np.complex128), D, mode="full")


class DDEKernels:
    """kernel_fn for operator.StackedOperator(..., extra_support=J_D - 1):
    Eq. (6) taps convolved with each visibility's D.

    ``d_u``, ``d_v``: complex [M, J_D] in the visibilities' order.  ``inner`` is
    the kernel function of the w-kernel itself (exact by default).
    """

    wants_index = True

    def __init__(self, d_u, d_v, inner=None):
        self.d_u = np.asarray(d_u, dtype=np.complex128)
        self.d_v = np.asarray(d_v, dtype=np.complex128)
        assert self.d_u.shape == self.d_v.shape and self.d_u.shape[1] % 2 == 1
        self.h = (self.d_u.shape[1] - 1) // 2
        self.inner = wkernel.visibility_kernel if inner is None else inner

    def __call__(self, u_pix, v_pix, w_eff, geom: Geometry, jp_total, p):
        u0, v0, K = self.inner(u_pix, v_pix, w_eff, geom, int(jp_total) - 2 * self.h)
        return u0 - self.h, v0 - self.h, convolve_kernel(K, self.d_u[p], self.d_v[p])


def support(w_eff, geom: Geometry, j_d: int):
    """J_p' = J_p + J_D - 1."""
    return wkernel.support(w_eff, geom) + (j_d - 1)
