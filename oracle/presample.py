"""Kernels interpolated from pre-sampled 1-D w-planes (Sec. 5.1.1).  FP64.

Test infrastructure only.

Radial symmetry makes the w-projection kernel a function of two variables,
the tap distance q (cells) and w, so it can be pre-sampled on a 2-D lattice
("1-D w-planes") and interpolated bilinearly instead of integrated per tap.
Only q, w >= 0 are sampled: K(q, -w) = conj K(q, w), and taps on either side
of the visibility see the same q.

    plane j:  w_j = j dw,   sample i:  q_i = i dq,   T[j, i] = K(q_i, w_j)  (Eq. (6))

At (q, w), with a = |w| / dw, j = floor(a), s = a - j and x = q / dq,
i = floor(x), t = x - i:

    K~(q, |w|) = (1 - s) [(1 - t) T[j, i] + t T[j, i+1]]
               +      s  [(1 - t) T[j+1, i] + t T[j+1, i+1]],
    K~(q, w)   = conj K~(q, |w|)  for w < 0.

The lattice is evaluated on demand (``PlaneSampler``): a plane's samples are
computed with the oracle's Eq. (6) quadrature the first time they are needed,
which is the same table as one computed in full beforehand.

Pins (tests/test_oracle_presample.py): a lattice filled from any bilinear
function a + b q + c w + d q w is reproduced exactly at every (q, w >= 0); at
the lattice nodes the interpolant equals the quadrature; the conjugate rule
for w < 0 against the direct kernel at -w; the error against the direct
kernel stays within the linear-interpolation bound h^2/8 max|f''| (second
derivatives measured on the direct kernel) and falls fourfold when both
steps are halved.
"""
from __future__ import annotations

import math

import numpy as np

from . import wkernel
from .wkernel import Geometry

# Steps that keep the interpolation error near 1e-4 of the kernel peak on the
# 25 degree workloads (linear-interpolation error ~0.22 dq^2 in q and up to
# ~0.02 dw^2 in w, relative to the peak).
DEFAULT_DQ = 1.0 / 64.0
DEFAULT_DW = 1.0 / 16.0


def bilinear(samples, q, w, dq: float, dw: float):
    """K~(q, w) from a lattice accessor ``samples(j, idx) -> T[j, idx]``.

    ``q`` is an array of distances (>= 0), ``w`` one scalar (any sign).
    """
    q = np.asarray(q, dtype=np.float64)
    aw = abs(float(w))
    a = aw / dw
    j = int(math.floor(a))
    s = a - j
    x = q / dq
    i = np.floor(x).astype(np.int64)
    t = x - i
    lo = (1.0 - t) * samples(j, i) + t * samples(j, i + 1)
    hi = (1.0 - t) * samples(j + 1, i) + t * samples(j + 1, i + 1)
    val = (1.0 - s) * lo + s * hi
    return np.conj(val) if w < 0 else val


class PlaneSampler:
    """T[j, i] = K(i dq, j dw) of Eq. (6), computed on first use.

    Samples are evaluated in fixed blocks of 512 consecutive indices per plane,
    so every value is independent of the order in which they are requested.
    """

    BLOCK = 512

    def __init__(self, geom: Geometry, dq: float = DEFAULT_DQ, dw: float = DEFAULT_DW):
        self.geom = geom
        self.dq = float(dq)
        self.dw = float(dw)
        self._blocks: dict[tuple, np.ndarray] = {}

    def __call__(self, j: int, idx):
        idx = np.asarray(idx, dtype=np.int64)
        out = np.empty(idx.shape, dtype=np.complex128)
        blk = idx // self.BLOCK
        for b in np.unique(blk):
            key = (j, int(b))
            vals = self._blocks.get(key)
            if vals is None:
                i0 = int(b) * self.BLOCK
                vals = wkernel.wkernel(np.arange(i0, i0 + self.BLOCK) * self.dq, j * self.dw,
                                       self.geom)
                self._blocks[key] = vals
            sel = blk == b
            out[sel] = vals[idx[sel] - int(b) * self.BLOCK]
        return out

    def kernel(self, q, w):
        """K~(q, w) for an array of distances q."""
        return bilinear(self, q, w, self.dq, self.dw)

    def visibility_kernel(self, u_pix: float, v_pix: float, w_eff: float, geom: Geometry,
                          jp: int | None = None):
        """(U0, V0, K~[J_p, J_p]): the taps of wkernel.visibility_kernel, interpolated."""
        if jp is None:
            jp = int(wkernel.support(w_eff, geom))
        u0, v0, q = wkernel.tap_geometry(u_pix, v_pix, jp)
        return u0, v0, self.kernel(q, w_eff)
