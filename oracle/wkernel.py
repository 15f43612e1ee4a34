"""Radial w-projection kernel of Eq. (6), support rule and tap geometry (FP64).

Test infrastructure only.

Conventions (Sec. 3.1, Eqs. (4)-(6)):

- image of N x N pixels of size dl = fov / N (direction cosine), padded by the
  oversampling factor alpha to a G x G Fourier grid, G = alpha N;
- Fourier cell du = 1 / (alpha N dl) = 1 / (alpha fov) wavelengths ("the
  resolution of the Fourier grid as determined by the zero padded field of
  view");
- a visibility at (u, v) sits at continuous grid coordinate
  (u_pix, v_pix) = (u, v) * (alpha fov);
- r is the image-domain radius in cycles per grid cell, r = rho du with
  rho = sqrt(l^2 + m^2), so sqrt(1 - r^2/du^2) = n.

Kernel (Eq. (6)), reading of the prefactor: with r in cycles per cell the
discrete tap weight is the continuous kernel times du^2, which turns the
paper's 2 pi / du^2 into 2 pi:

    K(q, w) = 2 pi int_0^{alpha/2} g(r) exp(-2 pi i w (n(r) - 1)) J0(2 pi r q) r dr,

q = distance (in cells) from (u_pix, v_pix) to the tap, w = w_p - wbar_k
(Eq. (5)).  The integral is evaluated by composite Gauss-Legendre quadrature
(a library rule) on panels that each hold at most half a cycle of the chirp
and at most half a cycle of J0(2 pi q r); the tests show that doubling the
panel count or switching to scipy's adaptive quadrature changes nothing above
1e-12 of the kernel peak.

Support rule (the paper only says the support shrinks as w - wbar shrinks,
Sec. 3.1): J_p = J + 2 ceil(|w| s), with s = rho_c / (n_c du) the chirp's
local frequency (cells per wavelength of w) at the image corner
rho_c = fov sqrt(1/2), n_c = sqrt(1 - rho_c^2), optionally multiplied by a
``support_scale`` f >= 1 (J_p = J + 2 ceil(|w| s f)).  The chirp's spectrum
has tails beyond its corner bandwidth, so f = 1 leaves a truncation error of
a few 1e-2 at 25 degrees for |w - wbar| ~ 10-40; larger f trades memory for
accuracy (the operator tests show the error falling to the w = 0 aliasing
level as f grows).  Taps are the J_p x J_p grid
points U0 .. U0 + J_p - 1 with U0 = floor(u_pix) - J_p/2 + 1 (and likewise
in v), taken modulo G (circular convolution, Sec. 2).

Pins (tests/test_oracle_wkernel.py): closed forms for g = 1 (q = 0 and w = 0),
a Gaussian taper with a paraxial chirp, w = 0 reducing to the KB blob,
K(q, -w) = conj K(q, w) (Sec. 5.1.1), a brute-force 2-D quadrature of the
un-reduced Fourier integral, and the local-frequency meaning of the support
rule.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy import special

from . import taper

GL_ORDER = 16


@dataclasses.dataclass(frozen=True)
class Geometry:
    n: int                       # image side (pixels), even
    fov: float                   # full field of view, radians (direction cosine)
    alpha: float = 2.0           # oversampling factor
    J: int = 4                   # KB support (cells), even
    beta: float | None = None    # KB shape; default 2.34 J
    max_support: int = 1024
    support_scale: float = 1.0   # multiplies the support slope s (1 = chirp band at the corner)

    def __post_init__(self):
        if self.n % 2:
            raise ValueError("image side must be even")
        if self.J % 2:
            raise ValueError("KB support must be even")
        g = self.alpha * self.n
        if abs(g - round(g)) > 1e-9 or int(round(g)) % 2:
            raise ValueError("alpha * n must be an even integer")
        if self.alpha * self.alpha * self.fov / 2.0 >= 1.0:
            raise ValueError("alpha^2 fov / 2 must be < 1 (horizon inside the kernel integral)")

    @property
    def kb_beta(self) -> float:
        return taper.default_beta(self.J) if self.beta is None else self.beta

    @property
    def grid_side(self) -> int:
        return int(round(self.alpha * self.n))

    @property
    def inv_du(self) -> float:
        """1 / du = alpha fov: multiply wavelengths by this to get grid cells."""
        return self.alpha * self.fov

    @property
    def du(self) -> float:
        return 1.0 / (self.alpha * self.fov)

    @property
    def r_max(self) -> float:
        return 0.5 * self.alpha

    @property
    def support_slope(self) -> float:
        rho_c = self.fov * math.sqrt(0.5)
        n_c = math.sqrt(1.0 - rho_c * rho_c)
        return (rho_c / (n_c * self.du)) * self.support_scale


def support(w_eff, geom: Geometry):
    """J_p = J + 2 ceil(|w_eff| s) (FP64 product, rounded once)."""
    w_eff = np.asarray(w_eff, dtype=np.float64)
    jp = geom.J + 2 * np.ceil(np.abs(w_eff) * geom.support_slope).astype(np.int64)
    return jp


def tap_geometry(u_pix: float, v_pix: float, jp: int):
    """Base indices and the distance q[row, col] from (u_pix, v_pix) to each tap."""
    u0 = int(math.floor(u_pix)) - jp // 2 + 1
    v0 = int(math.floor(v_pix)) - jp // 2 + 1
    du_ = u_pix - (u0 + np.arange(jp, dtype=np.float64))
    dv_ = v_pix - (v0 + np.arange(jp, dtype=np.float64))
    q = np.sqrt(dv_[:, None] ** 2 + du_[None, :] ** 2)
    return u0, v0, q


def panel_edges(r_max: float, q_max: float, breakpoints=()):
    n_uniform = max(1, int(math.ceil(r_max * (2.0 * q_max + 4.0))))
    edges = np.linspace(0.0, r_max, n_uniform + 1)
    bp = np.asarray(breakpoints, dtype=np.float64)
    bp = bp[(bp > 0.0) & (bp < r_max)]
    return np.unique(np.concatenate([edges, bp]))


def radial_transform(q, h, r_max: float, breakpoints=(), order: int = GL_ORDER,
                     refine: int = 1, chunk: int = 512):
    """2 pi int_0^{r_max} h(r) J0(2 pi q r) r dr for every q (composite Gauss-Legendre).

    ``h`` is a vectorised complex (or real) radial function; ``breakpoints``
    mark half cycles of its oscillation.  The q values are processed in
    ascending chunks, each on panels sized for that chunk's largest q.
    ``refine`` splits every panel into that many equal parts (used by the
    tests to show convergence).
    """
    q = np.asarray(q, dtype=np.float64)
    shape = q.shape
    qf = q.ravel()
    x, wgl = leggauss(order)
    order_idx = np.argsort(qf, kind="stable")
    out = None
    for s in range(0, qf.size, chunk):
        sel = order_idx[s:s + chunk]
        qc = qf[sel]
        edges = panel_edges(r_max, float(qc.max()), breakpoints)
        if refine > 1:
            fine = [np.linspace(a, b, refine + 1)[:-1] for a, b in zip(edges[:-1], edges[1:])]
            edges = np.concatenate(fine + [edges[-1:]])
        a = edges[:-1, None]
        b = edges[1:, None]
        half = 0.5 * (b - a)
        r = (half * x[None, :] + 0.5 * (a + b)).ravel()
        wr = (half * wgl[None, :]).ravel()
        hr = 2.0 * np.pi * np.asarray(h(r)) * r * wr
        if out is None:
            out = np.empty(qf.size, dtype=np.result_type(hr.dtype, np.float64))
        out[sel] = special.j0(2.0 * np.pi * np.outer(qc, r)) @ hr
    if out is None:
        out = np.empty(0)
    return out.reshape(shape)


def chirp_half_cycle_radii(w: float, geom: Geometry):
    """Radii where |w| (1 - n(r)) crosses k/2 cycles, k = 1, 2, ... (r < r_max)."""
    aw = abs(w)
    if aw == 0.0:
        return np.zeros(0)
    rho_end = geom.r_max / geom.du
    cyc_end = aw * (1.0 - math.sqrt(1.0 - rho_end * rho_end))
    k = np.arange(1, int(math.floor(2.0 * cyc_end)) + 1, dtype=np.float64)
    n = 1.0 - k / (2.0 * aw)
    return geom.du * np.sqrt(1.0 - n * n)


def chirp(r, w: float, geom: Geometry):
    """exp(-2 pi i w (n(r) - 1)), with n - 1 = -rho^2 / (1 + n), rho = r / du."""
    rho = np.asarray(r, dtype=np.float64) * geom.inv_du
    rho2 = rho * rho
    nm1 = -rho2 / (1.0 + np.sqrt(1.0 - rho2))
    return np.exp(-2j * np.pi * w * nm1)


def wkernel(q, w_eff: float, geom: Geometry, refine: int = 1):
    """K(q, w_eff) of Eq. (6) for an array of tap distances q (cells)."""
    def h(r):
        return taper.kb_blob_ft(r, geom.J, geom.kb_beta) * chirp(r, w_eff, geom)
    return radial_transform(q, h, geom.r_max, chirp_half_cycle_radii(w_eff, geom),
                            refine=refine)


def visibility_kernel(u_pix: float, v_pix: float, w_eff: float, geom: Geometry,
                      jp: int | None = None):
    """(U0, V0, K[J_p, J_p]) for one visibility; K[row, col] is tap (V0+row, U0+col)."""
    if jp is None:
        jp = int(support(w_eff, geom))
    u0, v0, q = tap_geometry(u_pix, v_pix, jp)
    return u0, v0, wkernel(q, w_eff, geom)
