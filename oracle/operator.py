"""The w-stacking w-projection measurement operator (FP64).  Test infrastructure only.

Eq. (2): Phi = W G C F Z S; Eq. (3): each w-stack k has
Phi_k = W_k GC_k F Z S~_k; Eq. (7): the adjoint sums the stacks' adjoints.

- S~_k (Eq. (4), a_k = 1): multiply pixel (j, i) by
  exp(-2 pi i wbar_k (n - 1)) / (g(r) n), r = rho du;
- Z: place the N x N image in a G x G array with pixel (N/2, N/2) at index
  (0, 0) (index (j - N/2) mod G, (i - N/2) mod G);
- F: unnormalised forward 2-D DFT, exp(-2 pi i), numpy.fft.fft2 (axis 0 = v,
  axis 1 = u);
- GC_k (Eq. (5)): y_p = sum_taps K_p[row, col] grid[(V0+row) mod G, (U0+col) mod G];
- W_k: real weights; a folded visibility (Eq. (8)) is returned conjugated.

Adjoint (real image, Eq. (2)'s x in R^N): gridding with conj(K), the
unnormalised inverse DFT (G^2 ifft2), crop, multiply by conj(S~_k), real
part, summed over stacks (Eq. (7)).

forward_at / adjoint_at evaluate the same operator with the stack grids
taken by the DFT's definition at only the cells (and image pixels) that a
subset of visibilities needs, for full-size problems.

Pins (tests/test_oracle_operator.py): agreement with the direct DFT of
Eq. (1) at the aliasing level; the adjoint dot-product identity to 1e-12;
independence of the number of stacks (Eq. (7)); folded vs unfolded agreement;
at w = 0, agreement with textbook separable Kaiser-Bessel gridding;
forward_at / adjoint_at equal to forward / adjoint (numpy FFT route) on
sparse and dense images.
"""
from __future__ import annotations

import numpy as np

from . import stacking, taper, wkernel
from .dft import n_minus_one, pixel_lm
from .wkernel import Geometry


def _correction(geom: Geometry, wbar: float, L, M):
    """S~_k (Eq. (4), no primary beam) at direction cosines (L, M)."""
    nm1, n = n_minus_one(L, M)
    r = np.sqrt(L * L + M * M) * geom.du
    g = taper.kb_blob_ft(r, geom.J, geom.kb_beta)
    return np.exp(-2j * np.pi * wbar * nm1) / (g * n)


def stack_correction(geom: Geometry, wbar: float):
    """S~_k as an [N, N] complex array (Eq. (4), no primary beam)."""
    lcol, mrow = pixel_lm(geom.n, geom.fov)
    L, M = np.meshgrid(lcol, mrow)
    return _correction(geom, wbar, L, M)


def stack_correction_at(geom: Geometry, wbar: float, rows, cols):
    """S~_k at pixels (rows, cols) only."""
    lcol, mrow = pixel_lm(geom.n, geom.fov)
    return _correction(geom, wbar, lcol[np.asarray(cols)], mrow[np.asarray(rows)])


_ROOTS = {}


def unit_roots(G: int):
    """exp(2 pi i k / G) for k = 0 .. G - 1 (the DFT's exponentials, by exact integer index)."""
    if G not in _ROOTS:
        _ROOTS[G] = np.exp(2j * np.pi * np.arange(G) / G)
    return _ROOTS[G]


def padded_index(geom: Geometry, idx):
    """Grid index that Z gives pixel row/column idx (pixel N/2 at index 0)."""
    return (np.asarray(idx, dtype=np.int64) - geom.n // 2) % geom.grid_side


def zero_pad(geom: Geometry, z):
    G, n = geom.grid_side, geom.n
    out = np.zeros((G, G), dtype=np.complex128)
    idx = (np.arange(n) - n // 2) % G
    out[np.ix_(idx, idx)] = z
    return out


def crop(geom: Geometry, big):
    G, n = geom.grid_side, geom.n
    idx = (np.arange(n) - n // 2) % G
    return big[np.ix_(idx, idx)]


class StackedOperator:
    """Phi for one set of visibilities, with a kernel per visibility (exact by default)."""

    def __init__(self, geom: Geometry, uvw, weights=None, n_stacks: int = 1,
                 fold: bool = False, labels=None, centres=None,
                 kmeans_tol: float = 1e-3, kmeans_max_iter: int = 100, kernel_fn=None,
                 extra_support: int = 0):
        self.geom = geom
        # (u_pix, v_pix, w_eff, geom, jp) -> (U0, V0, K): exact Eq. (6) taps by
        # default, or e.g. presample.PlaneSampler(...).visibility_kernel; a
        # function with ``wants_index`` set also gets the visibility's index
        # (keyword p).  extra_support widens every J_p (a DDE convolution).
        self.kernel_fn = wkernel.visibility_kernel if kernel_fn is None else kernel_fn
        uvw = np.asarray(uvw, dtype=np.float64)
        self.m = uvw.shape[0]
        if fold:
            uvw_f, self.flag = stacking.fold(uvw)
        else:
            uvw_f, self.flag = uvw.copy(), np.zeros(self.m, dtype=bool)
        self.uvw = uvw_f
        if labels is None:
            labels, centres, self.kmeans_iters = stacking.kmeans_w(
                uvw_f[:, 2], n_stacks, kmeans_tol, kmeans_max_iter)
        else:
            self.kmeans_iters = 0
        self.labels = np.asarray(labels, dtype=np.int64)
        self.centres = np.asarray(centres, dtype=np.float64)
        self.n_stacks = self.centres.size
        self.weights = (np.ones(self.m) if weights is None
                        else np.asarray(weights, dtype=np.float64))
        self.u_pix = uvw_f[:, 0] * geom.inv_du
        self.v_pix = uvw_f[:, 1] * geom.inv_du
        self.w_eff = uvw_f[:, 2] - self.centres[self.labels]
        self.jp = wkernel.support(self.w_eff, geom) + int(extra_support)
        self._kernels: dict[int, tuple] = {}

    def kernel(self, p: int):
        """(U0, V0, K[J_p, J_p]) of visibility p (cached)."""
        if p not in self._kernels:
            extra = {"p": p} if getattr(self.kernel_fn, "wants_index", False) else {}
            self._kernels[p] = self.kernel_fn(
                self.u_pix[p], self.v_pix[p], self.w_eff[p], self.geom, int(self.jp[p]), **extra)
        return self._kernels[p]

    def _stack_members(self, subset):
        idx = np.arange(self.m) if subset is None else np.asarray(subset)
        return [(k, idx[self.labels[idx] == k]) for k in range(self.n_stacks)]

    def stack_grid(self, x, k: int):
        """F Z S~_k x."""
        z = np.asarray(x, dtype=np.float64) * stack_correction(self.geom, self.centres[k])
        return np.fft.fft2(zero_pad(self.geom, z))

    def degrid_stack(self, grid, members, y):
        """W_k GC_k (Eq. (5)) for the visibilities ``members`` of one stack, from its grid; into y."""
        G = self.geom.grid_side
        for p in members:
            u0, v0, K = self.kernel(int(p))
            jp = K.shape[0]
            rows = (v0 + np.arange(jp)) % G
            cols = (u0 + np.arange(jp)) % G
            val = np.sum(K * grid[np.ix_(rows, cols)]) * self.weights[p]
            y[p] = np.conj(val) if self.flag[p] else val

    def forward(self, x, subset=None):
        """y = Phi x (all visibilities, or only ``subset``; others left 0)."""
        y = np.zeros(self.m, dtype=np.complex128)
        for k, members in self._stack_members(subset):
            if members.size == 0:
                continue
            self.degrid_stack(self.stack_grid(x, k), members, y)
        return y

    def _subset_taps(self, members):
        """Grid cells (V, U) and values K of the taps of ``members``, and each tap's position in ``members``."""
        G = self.geom.grid_side
        rows, cols, vals, owner = [], [], [], []
        for pos, p in enumerate(members):
            u0, v0, K = self.kernel(int(p))
            jp = K.shape[0]
            r = (v0 + np.arange(jp)) % G
            c = (u0 + np.arange(jp)) % G
            rows.append(np.repeat(r, jp))
            cols.append(np.tile(c, jp))
            vals.append(K.ravel())
            owner.append(np.full(jp * jp, pos, dtype=np.int64))
        return (np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), np.concatenate(owner))

    def forward_at(self, x, subset, chunk: int = 2048):
        """y = Phi x on the visibilities ``subset`` only (others 0), like forward().

        Each stack grid F Z S~_k x is evaluated by the DFT's definition at just
        the cells the subset's taps touch:
            grid[V, U] = sum_{j, i} z[j, i] exp(-2 pi i (U U_i + V V_j) / G),
        z = x S~_k, (V_j, U_i) the position Z gives pixel (j, i), summed over
        the non-zero pixels of x (the exponent's integer part reduced mod G
        exactly).  The cost scales with the non-zero pixels times the touched
        cells, so full-size grids need no G x G transform."""
        G = self.geom.grid_side
        x = np.asarray(x, dtype=np.float64)
        jj, ii = np.nonzero(x)
        Vp, Up = padded_index(self.geom, jj), padded_index(self.geom, ii)
        y = np.zeros(self.m, dtype=np.complex128)
        for k, members in self._stack_members(subset):
            if members.size == 0:
                continue
            z = x[jj, ii] * stack_correction_at(self.geom, self.centres[k], jj, ii)
            rows, cols, vals, owner = self._subset_taps(members)
            cell = rows * G + cols
            uniq, inv = np.unique(cell, return_inverse=True)
            V, U = uniq // G, uniq % G
            gv = np.empty(uniq.size, dtype=np.complex128)
            for s in range(0, uniq.size, chunk):
                m_ = (U[s:s + chunk, None] * Up[None, :] + V[s:s + chunk, None] * Vp[None, :]) % G
                gv[s:s + chunk] = np.conj(unit_roots(G)[m_]) @ z
            contrib = vals * gv[inv]
            sums = (np.bincount(owner, weights=contrib.real, minlength=members.size)
                    + 1j * np.bincount(owner, weights=contrib.imag, minlength=members.size))
            for p, val in zip(members, sums):
                val = val * self.weights[p]
                y[p] = np.conj(val) if self.flag[p] else val
        return y

    def adjoint_at(self, y, rows, cols, subset, chunk: int = 2048):
        """x = Re Phi^dagger y at pixels (rows, cols) only, for y non-zero only on ``subset``.

        Each stack's gridded cells (conj(K) W y of the subset's taps, summed
        per cell) are taken to the pixels by the unnormalised inverse DFT's
        definition, sum_cells grid[V, U] exp(+2 pi i (U U_i + V V_j) / G), then
        multiplied by conj(S~_k), the real part taken and the stacks summed
        (Eq. (7)), like adjoint()."""
        G = self.geom.grid_side
        rows = np.asarray(rows, dtype=np.int64)
        cols = np.asarray(cols, dtype=np.int64)
        Vp, Up = padded_index(self.geom, rows), padded_index(self.geom, cols)
        y = np.asarray(y, dtype=np.complex128)
        out = np.zeros(rows.size)
        subset = np.asarray(subset)
        for k, members in self._stack_members(subset):
            if members.size == 0:
                continue
            r_, c_, vals, pos = self._subset_taps(members)
            owner = members[pos]
            yp = np.where(self.flag[owner], np.conj(y[owner]), y[owner]) * self.weights[owner]
            contrib = np.conj(vals) * yp
            cell = r_ * G + c_
            uniq, inv = np.unique(cell, return_inverse=True)
            gv = (np.bincount(inv, weights=contrib.real, minlength=uniq.size)
                  + 1j * np.bincount(inv, weights=contrib.imag, minlength=uniq.size))
            V, U = uniq // G, uniq % G
            acc = np.zeros(rows.size, dtype=np.complex128)
            for s in range(0, uniq.size, chunk):
                m_ = (U[s:s + chunk, None] * Up[None, :] + V[s:s + chunk, None] * Vp[None, :]) % G
                acc += gv[s:s + chunk] @ unit_roots(G)[m_]
            out += np.real(np.conj(stack_correction_at(self.geom, self.centres[k], rows, cols)) * acc)
        return out

    def grid_stack(self, y, members):
        """(W_k GC_k)^dagger: the stack's G x G grid of conj(K) W y over ``members``."""
        G = self.geom.grid_side
        y = np.asarray(y, dtype=np.complex128)
        grid = np.zeros((G, G), dtype=np.complex128)
        for p in members:
            u0, v0, K = self.kernel(int(p))
            jp = K.shape[0]
            yp = np.conj(y[p]) if self.flag[p] else y[p]
            rows = (v0 + np.arange(jp)) % G
            cols = (u0 + np.arange(jp)) % G
            np.add.at(grid, np.ix_(rows, cols), np.conj(K) * (self.weights[p] * yp))
        return grid

    def finish_adjoint(self, grid, k: int):
        """Re S~_k^dagger Z^dagger F^dagger of one stack's grid (its term of Eq. (7))."""
        G = self.geom.grid_side
        big = np.fft.ifft2(grid) * (G * G)
        return np.real(np.conj(stack_correction(self.geom, self.centres[k])) * crop(self.geom, big))

    def adjoint(self, y, subset=None):
        """x = Re Phi^dagger y summed over stacks (Eq. (7))."""
        x = np.zeros((self.geom.n, self.geom.n))
        for k, members in self._stack_members(subset):
            if members.size == 0:
                continue
            x += self.finish_adjoint(self.grid_stack(y, members), k)
        return x


def separable_kb_forward(geom: Geometry, x, uvw):
    """Textbook separable KB gridding at w = 0 (second route for the w = 0 check).

    Correction 1 / (G1(l du) G1(m du) n) with the 1-D KB transform G1, taps
    k1(du_col) k1(dv_row) on the J x J nearest grid points; the w-term is
    ignored.
    """
    G = geom.grid_side
    J, beta = geom.J, geom.kb_beta
    lcol, mrow = pixel_lm(geom.n, geom.fov)
    L, M = np.meshgrid(lcol, mrow)
    _, n = n_minus_one(L, M)
    corr = 1.0 / (taper.kb_1d_ft(L * geom.du, J, beta) * taper.kb_1d_ft(M * geom.du, J, beta) * n)
    grid = np.fft.fft2(zero_pad(geom, np.asarray(x, dtype=np.float64) * corr))
    uvw = np.asarray(uvw, dtype=np.float64)
    y = np.empty(uvw.shape[0], dtype=np.complex128)
    for p in range(uvw.shape[0]):
        up, vp = uvw[p, 0] * geom.inv_du, uvw[p, 1] * geom.inv_du
        u0 = int(np.floor(up)) - J // 2 + 1
        v0 = int(np.floor(vp)) - J // 2 + 1
        cu = u0 + np.arange(J)
        cv = v0 + np.arange(J)
        K = np.outer(taper.kb_1d(vp - cv, J, beta), taper.kb_1d(up - cu, J, beta))
        y[p] = np.sum(K * grid[np.ix_(cv % G, cu % G)])
    return y
