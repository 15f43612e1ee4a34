"""The all-FP64 GPU path at the benchmark's geometry: kernel taps at large w.

The tiny parity case keeps 2 pi r q below ~30; on the 1024^2, 25 deg MWA-like
track the Bessel argument reaches ~1e3 and |w - wbar| ~250, which exercises
the FP64 Hankel branch and the FP64 phase reductions of the FP64 tap kernel.
A handful of visibilities of that track, up to the largest support, are
built on the FP64 path; on each, a seeded sample of taps (with the smallest
and the largest distance q) is compared with the oracle.
"""
import math

import numpy as np
import pytest

from oracle import operator, wkernel
from paper_1903_06555_amd import synthetic as syn
from paper_1903_06555_amd import wsp

pytestmark = pytest.mark.gpu


def test_fp64_kernels_large_w():
    wl = syn.WORKLOADS["mwa_1024_single_stack"]
    uvw = syn.workload_uvw(wl)
    geom = wkernel.Geometry(n=wl.n, fov=math.radians(wl.fov_deg))
    w = uvw[:, 2]
    centre = 0.5 * (w.min() + w.max())
    jp = wkernel.support(w - centre, geom)
    order = np.argsort(jp, kind="stable")
    pick = np.unique(order[(np.array([0.1, 0.5, 0.9, 0.999, 1.0]) * (len(order) - 1)).astype(int)])
    sub = uvw[pick]
    labels = np.zeros(len(pick), dtype=np.int32)
    centres = np.array([centre])
    ref = operator.StackedOperator(geom, sub, labels=labels, centres=centres)
    params = wsp.make_params(wl.n, geom.fov, n_stacks=1, precision="fp64")
    op = wsp.Operator(params, sub, labels=labels, centres=centres)
    rng = np.random.default_rng(17)
    try:
        assert np.array_equal(op.support()[0], ref.jp)
        assert ref.jp.max() == jp.max()
        for p in range(len(pick)):
            K, u0, v0 = op.kernel(p)
            # the oracle on a seeded sample of taps, always with the smallest and largest q
            ru0, rv0, q = wkernel.tap_geometry(ref.u_pix[p], ref.v_pix[p], int(ref.jp[p]))
            assert (u0, v0) == (ru0, rv0)
            qf = q.ravel()
            sel = np.unique(np.concatenate([rng.choice(qf.size, min(qf.size, 3000), replace=False),
                                            [np.argmin(qf), np.argmax(qf)]]))
            Kr = wkernel.wkernel(qf[sel], float(ref.w_eff[p]), geom)
            Kg = K.ravel()[sel]
            err = float(np.max(np.abs(Kg - Kr)) / np.max(np.abs(Kr)))
            print(f"J_p {K.shape[0]} |w_eff| {abs(ref.w_eff[p]):.1f} ({sel.size} taps): "
                  f"max|dK|/max|K| = {err:.2e}", flush=True)
            assert err <= 1e-6
    finally:
        op.close()
