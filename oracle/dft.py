"""Direct evaluation of the measurement equation (FP64).  Test infrastructure only.

Eq. (1) of the paper with no direction-dependent term (a = 1, the choice
stated for the stacks in Sec. 3.1), evaluated as a sum over image pixels:

    y_p = W_p sum_{j,i} x[j, i] exp(-2 pi i w_p (n_ji - 1)) / n_ji
                               * exp(-2 pi i (u_p l_i + v_p m_j)),

with n = sqrt(1 - l^2 - m^2), l_i = (i - N/2) dl, m_j = (j - N/2) dl,
dl = fov / N (row j <-> m, column i <-> l, phase centre on pixel N/2).
x is in Jy per pixel, so no dl dm factor is applied.  The raw w of each
visibility is used: the global mean w of Eq. (1) is subsumed by the stacks.

The adjoint (for a real image, Eq. (2)'s x in R^N) is

    x[j, i] = Re sum_p conj(phase_p(j, i)) W_p y_p.

Pins (tests/test_oracle_dft.py): the phase equals -2 pi times the
baseline-direction dot product b . (s - s0); the w = 0 case equals numpy's
FFT at integer frequencies; conjugate symmetry Eq. (8); the adjoint
dot-product identity.
"""
from __future__ import annotations

import numpy as np


def pixel_lm(n: int, fov: float):
    """Direction cosines (l of columns, m of rows) of an n x n image."""
    dl = fov / n
    idx = (np.arange(n) - n // 2).astype(np.float64)
    return idx * dl, idx * dl


def n_minus_one(l, m):
    """n - 1 = -rho^2 / (1 + n), written to avoid cancellation near the centre."""
    rho2 = l * l + m * m
    n = np.sqrt(1.0 - rho2)
    return -rho2 / (1.0 + n), n


def _phases(uvw, l, m):
    nm1, n = n_minus_one(l, m)
    u, v, w = uvw[:, 0:1], uvw[:, 1:2], uvw[:, 2:3]
    arg = u * l[None, :] + v * m[None, :] + w * nm1[None, :]
    return np.exp(-2j * np.pi * arg) / n[None, :]


def measure(x, uvw, fov: float, weights=None, chunk: int = 256):
    """y = Phi_DFT x for a real image x [N, N]; returns complex128 [M]."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    lcol, mrow = pixel_lm(n, fov)
    jj, ii = np.nonzero(x)
    vals = x[jj, ii]
    l = lcol[ii]
    m = mrow[jj]
    uvw = np.asarray(uvw, dtype=np.float64)
    y = np.empty(uvw.shape[0], dtype=np.complex128)
    for s in range(0, uvw.shape[0], chunk):
        y[s:s + chunk] = _phases(uvw[s:s + chunk], l, m) @ vals
    if weights is not None:
        y *= np.asarray(weights, dtype=np.float64)
    return y


def measure_adjoint(y, uvw, n: int, fov: float, weights=None, chunk: int = 256):
    """x = Re Phi_DFT^dagger y, real [N, N]."""
    y = np.asarray(y, dtype=np.complex128)
    if weights is not None:
        y = y * np.asarray(weights, dtype=np.float64)
    lcol, mrow = pixel_lm(n, fov)
    L, Mm = np.meshgrid(lcol, mrow)
    l = L.ravel()
    m = Mm.ravel()
    acc = np.zeros(l.size, dtype=np.complex128)
    uvw = np.asarray(uvw, dtype=np.float64)
    for s in range(0, uvw.shape[0], chunk):
        acc += np.conj(_phases(uvw[s:s + chunk], l, m)).T @ y[s:s + chunk]
    return acc.real.reshape(n, n)
