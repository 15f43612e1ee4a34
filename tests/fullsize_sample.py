"""Stratified visibility samples for the full-size parity tests (test infrastructure).

From the oracle's own geometry (pixel coordinates, supports, stacks) it picks,
in every w-stack, visibilities at uniform quantiles of the support J_p
(largest included), and adds visibilities of three kinds the tile kernels
treat specially:

- seam: the J_p x J_p footprint covers grid index G - 1 and 0 in u or v,
  so it wraps across the grid's edge (Eq. (2)'s circular convolution);
- aliased: the visibility lies beyond the grid's half-width in u or v;
- split: a footprint entry falls in a 64 x 64 tile holding more taps than
  one work item, so the tile is split over several items (the item cut
  happens inside the tile's entry list).
"""
from __future__ import annotations

import numpy as np

TILE = 64
ITEM_TAPS = 1 << 19


def tile_taps(ref):
    """Taps per (stack, tile) and, per visibility, its footprint's tile keys (-1: none)."""
    G = ref.geom.grid_side
    nt = G // TILE
    jp = ref.jp.astype(np.int64)
    u0 = (np.floor(ref.u_pix).astype(np.int64) - jp // 2 + 1) % G
    v0 = (np.floor(ref.v_pix).astype(np.int64) - jp // 2 + 1) % G
    keys, counts = [], []
    for dy in range(0, int(jp.max()) // TILE + 2):
        for dx in range(0, int(jp.max()) // TILE + 2):
            tvx = u0 // TILE + dx
            tvy = v0 // TILE + dy
            c0 = np.maximum(tvx * TILE - u0, 0)
            c1 = np.minimum((tvx + 1) * TILE - u0, jp)
            r0 = np.maximum(tvy * TILE - v0, 0)
            r1 = np.minimum((tvy + 1) * TILE - v0, jp)
            n = np.where((c1 > c0) & (r1 > r0), (c1 - c0) * (r1 - r0), 0)
            key = (ref.labels.astype(np.int64) * nt + tvy % nt) * nt + tvx % nt
            keys.append(np.where(n > 0, key, -1))
            counts.append(n)
    keys = np.stack(keys, 1)
    counts = np.stack(counts, 1)
    total = np.bincount(keys[keys >= 0], weights=counts[keys >= 0],
                        minlength=int(ref.n_stacks) * nt * nt)
    return total, keys


def sample(ref, per_stack: int, extra: int, seed: int):
    """Sorted unique visibility indices, and a dict of the special kinds found."""
    G = ref.geom.grid_side
    rng = np.random.default_rng(seed)
    picks = []
    for k in range(ref.n_stacks):
        members = np.flatnonzero(ref.labels == k)
        if members.size == 0:
            continue
        order = members[np.argsort(ref.jp[members], kind="stable")]
        q = np.unique(np.linspace(0, order.size - 1, min(per_stack, order.size)).astype(np.int64))
        picks.append(order[q])
    jp = ref.jp.astype(np.int64)
    U0 = np.floor(ref.u_pix).astype(np.int64) - jp // 2 + 1
    V0 = np.floor(ref.v_pix).astype(np.int64) - jp // 2 + 1
    seam = np.flatnonzero(((U0 % G) + jp > G) | ((V0 % G) + jp > G))
    aliased = np.flatnonzero((np.abs(ref.u_pix) > G / 2) | (np.abs(ref.v_pix) > G / 2))
    total, keys = tile_taps(ref)
    big = np.flatnonzero(total > ITEM_TAPS + int(jp.max()) ** 2)
    split = np.flatnonzero(np.isin(keys, big).any(axis=1)) if big.size else np.zeros(0, np.int64)
    kinds = {}
    for name, idx in (("seam", seam), ("aliased", aliased), ("split", split)):
        kinds[name] = int(idx.size)
        if idx.size:
            picks.append(rng.choice(idx, size=min(extra, idx.size), replace=False))
    return np.unique(np.concatenate(picks)), kinds


def pixels(n: int, count: int, seed: int):
    """Image pixels (rows, cols): corners, edge midpoints, centre, and random ones."""
    rng = np.random.default_rng(seed)
    fixed = [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1), (n // 2, n // 2), (0, n // 2),
             (n // 2, 0), (n - 1, n // 2), (n // 2, n - 1)]
    rows = np.concatenate([[r for r, _ in fixed], rng.integers(0, n, count)])
    cols = np.concatenate([[c for _, c in fixed], rng.integers(0, n, count)])
    return rows, cols
