"""Write tests/golden/fullsize_1024.npz: oracle values for the 1024^2 full-size parity test.

Calls only the oracle (oracle/) and the seeded input generators; nothing
here touches the GPU library.  The workload is the 1024^2, 25 degree,
1e6-visibility single-stack MWA-like set (synthetic.WORKLOADS
["mwa_1024_single_stack"]).  The sample (tests/fullsize_sample.py, seed 62)
holds 200 visibilities at uniform quantiles of J_p up to the largest (282)
plus footprints across the grid's edge, aliased and split-tile ones; its
exact kernels (Eq. (6)) take about half an hour of one core, so they are
computed here once, by a process pool, instead of inside the GPU test.

Stored: the sample and its supports; y = Phi x of the workload sky on the
sample (every sampled value); x = Re Phi^dagger y for y non-zero only on the
sample (random_vis(sample.size, 31)) at 2057 pixels; and per sampled
visibility 64 taps (the 3 x 3 around the visibility, the four corners and
55 at random) with their positions and the kernel's peak magnitude.

    python tests/golden/make_fullsize_1024.py
"""
from __future__ import annotations

import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import fullsize_sample  # noqa: E402
import oracle_pool  # noqa: E402
from oracle import operator, wkernel  # noqa: E402
from paper_1903_06555_amd import synthetic as syn  # noqa: E402

OUT = os.path.join(HERE, "fullsize_1024.npz")
TAPS_PER_VIS = 64


def tap_positions(ref, p, rng):
    jp = int(ref.jp[p])
    u0, v0, _ = wkernel.tap_geometry(ref.u_pix[p], ref.v_pix[p], jp)
    cr, cc = int(math.floor(ref.v_pix[p])) - v0, int(math.floor(ref.u_pix[p])) - u0
    pos = {(r, c) for r in (cr - 1, cr, cr + 1) for c in (cc - 1, cc, cc + 1) if 0 <= r < jp and 0 <= c < jp}
    pos |= {(0, 0), (0, jp - 1), (jp - 1, 0), (jp - 1, jp - 1)}
    while len(pos) < min(TAPS_PER_VIS, jp * jp):
        pos.add((int(rng.integers(jp)), int(rng.integers(jp))))
    pos = sorted(pos)[:TAPS_PER_VIS]
    while len(pos) < TAPS_PER_VIS:  # tiny supports: repeat the first position
        pos.append(pos[0])
    return np.array(pos, dtype=np.int32)


def main():
    wl = syn.WORKLOADS["mwa_1024_single_stack"]
    uvw = syn.workload_uvw(wl)
    x = syn.workload_sky(wl)
    geom = wkernel.Geometry(n=wl.n, fov=math.radians(wl.fov_deg))
    ref = operator.StackedOperator(geom, uvw, n_stacks=1)
    sample, kinds = fullsize_sample.sample(ref, 200, 12, seed=62)
    print(f"{sample.size} visibilities, kinds {kinds}", flush=True)
    oracle_pool.fill_kernels(ref, sample)
    y_ref = ref.forward(x, subset=sample)[sample]
    yin = np.zeros(ref.m, dtype=np.complex128)
    yin[sample] = syn.random_vis(sample.size, seed=31)
    rows, cols = fullsize_sample.pixels(wl.n, 2048, seed=32)
    x_ref = ref.adjoint(yin, subset=sample)[rows, cols]
    rng = np.random.default_rng(63)
    pos = np.zeros((sample.size, TAPS_PER_VIS, 2), dtype=np.int32)
    taps = np.zeros((sample.size, TAPS_PER_VIS), dtype=np.complex128)
    peak = np.zeros(sample.size)
    for i, p in enumerate(sample):
        _, _, K = ref.kernel(int(p))
        pos[i] = tap_positions(ref, int(p), rng)
        taps[i] = K[pos[i, :, 0], pos[i, :, 1]]
        peak[i] = np.max(np.abs(K))
    np.savez_compressed(OUT, sample=sample, jp=ref.jp[sample].astype(np.int32), y_ref=y_ref,
                        rows=rows, cols=cols, x_ref=x_ref, tap_pos=pos, taps=taps, peak=peak)
    print("wrote", OUT, os.path.getsize(OUT), "bytes")


if __name__ == "__main__":
    main()
