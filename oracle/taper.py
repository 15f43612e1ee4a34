"""Anti-aliasing taper pairs (FP64).  Test infrastructure only.

The paper names a "radial anti-aliasing filter" g (Eq. (4) divides the image
by it, Eq. (6) integrates it against the w-chirp) without giving its form.
Reading used here: g is the exact two-dimensional Fourier transform of the
radial Kaiser-Bessel "blob"

    k(q) = I0(beta sqrt(1 - (q/a)^2)) / I0(beta),   q < a = J/2 (grid cells),

which is (Lewitt 1990, JOSA A 7, 1834, n = 2, m = 0)

    g(r) = 2 pi a^2 / I0(beta) * I1(z) / z,   z = sqrt(beta^2 - (2 pi a r)^2),

continued as J1(z') / z' with z' = sqrt((2 pi a r)^2 - beta^2) past the main
lobe, and 1/2 at z = 0.  r is in cycles per padded-grid cell.  With this
pair the w = 0 kernel of Eq. (6) is the blob itself (up to truncation of the
integral at r = alpha/2).

Also provided: the separable one-dimensional Kaiser-Bessel pair of textbook
gridding, used only as a second route to the w = 0 operator.

Pins (tests/test_oracle_taper.py): numerical Hankel transform of k against
the closed form g; numerical 1-D Fourier transform of the 1-D window against
its closed form.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def default_beta(J: int) -> float:
    """Kaiser-Bessel shape 2.34 J (Fessler & Sutton 2003, for 2x oversampling)."""
    return 2.34 * J


def kb_blob(q, J: int, beta: float):
    """Radial KB blob k(q) in grid cells; zero for q >= J/2."""
    q = np.asarray(q, dtype=np.float64)
    a = 0.5 * J
    t = 1.0 - (q / a) ** 2
    inside = t > 0.0
    out = np.zeros_like(q)
    out[inside] = special.i0(beta * np.sqrt(t[inside])) / special.i0(beta)
    return out


def kb_blob_ft(r, J: int, beta: float):
    """g(r): exact 2-D Fourier transform of ``kb_blob`` at radius r (cycles/cell)."""
    r = np.asarray(r, dtype=np.float64)
    a = 0.5 * J
    z2 = beta * beta - (2.0 * np.pi * a * r) ** 2
    ratio = np.full_like(r, 0.5)
    pos = z2 > 0.0
    neg = z2 < 0.0
    z = np.sqrt(z2[pos])
    ratio[pos] = special.i1(z) / z
    zn = np.sqrt(-z2[neg])
    ratio[neg] = special.j1(zn) / zn
    return 2.0 * np.pi * a * a / special.i0(beta) * ratio


def kb_1d(x, J: int, beta: float):
    """Separable 1-D KB window on |x| < J/2 (grid cells)."""
    x = np.asarray(x, dtype=np.float64)
    t = 1.0 - (2.0 * x / J) ** 2
    out = np.zeros_like(x)
    inside = t > 0.0
    out[inside] = special.i0(beta * np.sqrt(t[inside])) / special.i0(beta)
    return out


def kb_1d_ft(r, J: int, beta: float):
    """Exact 1-D Fourier transform of ``kb_1d`` at frequency r (cycles/cell)."""
    r = np.asarray(r, dtype=np.float64)
    s2 = beta * beta - (np.pi * J * r) ** 2
    out = np.full_like(r, 1.0)
    pos = s2 > 0.0
    neg = s2 < 0.0
    s = np.sqrt(s2[pos])
    out[pos] = np.sinh(s) / s
    sn = np.sqrt(-s2[neg])
    out[neg] = np.sin(sn) / sn
    return J * out / special.i0(beta)
