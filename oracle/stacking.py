"""Conjugate-symmetry folding (Eq. (8)) and k-means w-stacking (Algorithm 1).

Test infrastructure only.  FP64, sums in visibility order.

Readings of Algorithm 1 (Sec. 3.2), where the printed pseudocode is
ambiguous or inconsistent:

- the per-visibility minimum starts at +inf (the printed 2 (w_max - w_min)
  is compared against a squared distance and would drop visibilities);
- ties go to the lowest stack index (strict "<" in stack order);
- an empty stack gets centre 0, as printed;
- initial centres: w_min + q (w_max - w_min) / (K - 1), q = 0..K-1, with the
  last set exactly to w_max; K = 1 starts at (w_min + w_max) / 2;
- convergence (Sec. 4: "average relative difference ... less than 1e-3"):
  mean_q |c_new - c_old| / max(|c_new|, 1e-12 max(w_max - w_min, 1)) < tol,
  capped at ``max_iter`` iterations;
- the returned labels are those of the last assignment pass and the returned
  centres their means.

Folding (Sec. 3.3): a visibility with w < 0 (strictly) is replaced by
(-u, -v, -w) and flagged; its model value is the complex conjugate of the
folded one (Eq. (8)), and in the adjoint its datum enters conjugated.

Pins (tests/test_oracle_stacking.py): brute-force Lloyd fixed point on tiny
inputs, monotone within-stack sum of squares, exact fold identity on the
operator output.
"""
from __future__ import annotations

import numpy as np


def fold(uvw):
    """Return (folded uvw, flag) with flag[p] = True where w_p < 0."""
    uvw = np.asarray(uvw, dtype=np.float64)
    flag = uvw[:, 2] < 0.0
    out = uvw.copy()
    out[flag] = -out[flag]
    return out, flag


def initial_centres(wmin: float, wmax: float, k: int):
    if k == 1:
        return np.array([0.5 * (wmin + wmax)])
    step = (wmax - wmin) / (k - 1)
    c = np.arange(k, dtype=np.float64) * step + wmin
    c[-1] = wmax
    return c


def assign(w, centres):
    """Nearest centre, strict '<' so that ties keep the lowest index."""
    best = np.full(w.shape, np.inf)
    label = np.zeros(w.shape, dtype=np.int64)
    for q, c in enumerate(centres):
        d = (c - w) ** 2
        better = d < best
        best[better] = d[better]
        label[better] = q
    return label


def update(w, labels, k: int):
    # bincount accumulates sequentially in visibility order
    wsum = np.bincount(labels, weights=w, minlength=k).astype(np.float64)
    wcount = np.bincount(labels, minlength=k).astype(np.int64)
    centres = np.zeros(k)
    nz = wcount > 0
    centres[nz] = wsum[nz] / wcount[nz]
    return centres, wcount


def kmeans_w(w, k: int, tol: float = 1e-3, max_iter: int = 100):
    """Algorithm 1.  Returns (labels int64[M], centres float64[K], iterations)."""
    w = np.asarray(w, dtype=np.float64)
    wmin, wmax = float(w.min()), float(w.max())
    centres = initial_centres(wmin, wmax, k)
    floor = 1e-12 * max(wmax - wmin, 1.0)
    labels = np.zeros(w.shape, dtype=np.int64)
    it = 0
    for it in range(1, max_iter + 1):
        labels = assign(w, centres)
        new, _ = update(w, labels, k)
        rel = np.mean(np.abs(new - centres) / np.maximum(np.abs(new), floor))
        centres = new
        if rel < tol:
            break
    return labels, centres, it


def within_stack_sse(w, labels, centres):
    return float(np.sum((np.asarray(w) - np.asarray(centres)[labels]) ** 2))
