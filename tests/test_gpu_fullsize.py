"""GPU parity at the benchmark's full size, in the benchmark's launch configuration.

Workload: 1024^2 image, 25 deg, 1e6 MWA-like visibilities, one w-stack,
FP32 data with FP64 phases (mean J_p 87, max 282, 88 GB of taps; most tiles
split over many work items).  The oracle cannot evaluate a million kernels,
so it checks, element by element, a sample of more than 200 visibilities:
200 at uniform quantiles of J_p (the largest included) plus visibilities
whose footprint wraps across the grid's edge, visibilities beyond the grid's
half-width (aliased by the circular convolution) and visibilities in split
tiles (tests/fullsize_sample.py).  The sample's exact oracle kernels take
about half an hour of one core, so its oracle values were written once by
tests/golden/make_fullsize_1024.py (oracle only) into
tests/golden/fullsize_1024.npz: every sampled degridded value of the
workload sky, the gridded image at 2057 pixels for an input non-zero only on
the sample, and 64 taps plus the peak of every sampled kernel.  The test
re-derives the sample and the supports from the oracle and checks they match
the stored ones.  The adjoint identity is checked on the whole operator.

Bars: taps max|dK| / max|K| <= 1e-6 per visibility; degrid
max_p |dy_p| / max|y| <= 1e-5 over the sample; grid max|dx| / max|x| <= 1e-5
over the stored pixels; the FP32 adjoint identity <= 1e-6.
"""
import math
import os

import numpy as np
import pytest
import torch

import adjoint_check
import fullsize_sample
from oracle import operator, wkernel
from paper_1903_06555_amd import synthetic as syn
from paper_1903_06555_amd import wsp

pytestmark = pytest.mark.gpu


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_1024.npz")


@pytest.fixture(scope="module")
def full():
    wl = syn.WORKLOADS["mwa_1024_single_stack"]
    uvw = syn.workload_uvw(wl)
    x = syn.workload_sky(wl)
    geom = wkernel.Geometry(n=wl.n, fov=math.radians(wl.fov_deg))
    ref = operator.StackedOperator(geom, uvw, n_stacks=1)
    gold = dict(np.load(GOLDEN, allow_pickle=False))
    sample, kinds = fullsize_sample.sample(ref, 200, 12, seed=62)
    assert np.array_equal(sample, gold["sample"]) and np.array_equal(ref.jp[sample], gold["jp"])
    params = wsp.make_params(wl.n, geom.fov, n_stacks=1, precision=wl.precision)
    op = wsp.Operator(params, uvw, labels=ref.labels, centres=ref.centres, build=False)
    op.build(part=200_000, progress=lambda d, n: print(f"built {d}/{n}", flush=True))
    st = op.plan_stats()
    print(f"{sample.size} sampled, J_p {ref.jp[sample].min()}-{ref.jp[sample].max()}, kinds {kinds}; "
          f"plan: {st['items']} items, {st['split_tiles']} split tiles", flush=True)
    yield wl, uvw, x, ref, op, sample, gold
    op.close()


def test_sample_covers_kinds(full):
    wl, uvw, x, ref, op, sample, gold = full
    assert sample.size >= 200
    G = ref.geom.grid_side
    assert np.any((np.abs(ref.u_pix[sample]) > G / 2) | (np.abs(ref.v_pix[sample]) > G / 2))
    assert ref.jp[sample].max() == ref.jp.max()


def test_supports_bit_exact(full):
    wl, uvw, x, ref, op, sample, gold = full
    jp, folded = op.support()
    assert np.array_equal(jp, ref.jp)
    assert not folded.any()


def test_sampled_kernels(full):
    wl, uvw, x, ref, op, sample, gold = full
    worst = 0.0
    for i, p in enumerate(sample):
        K, u0, v0 = op.kernel(int(p))
        ru0, rv0, _ = wkernel.tap_geometry(ref.u_pix[p], ref.v_pix[p], int(ref.jp[p]))
        assert (u0, v0) == (ru0, rv0) and K.shape == (ref.jp[p], ref.jp[p])
        pos = gold["tap_pos"][i]
        err = float(np.max(np.abs(K[pos[:, 0], pos[:, 1]] - gold["taps"][i])) / gold["peak"][i])
        err = max(err, abs(float(np.max(np.abs(K))) - gold["peak"][i]) / gold["peak"][i])
        assert err <= 1e-6, (int(p), int(ref.jp[p]), err)
        worst = max(worst, err)
    print(f"worst tap error over {sample.size} visibilities {worst:.2e}", flush=True)


def test_sampled_degrid(full):
    wl, uvw, x, ref, op, sample, gold = full
    # every per-run partial must come from this call: poison the scratch
    op.scratch.fill_(255)
    y = op.degrid(torch.from_numpy(x)).cpu().numpy()
    assert np.isfinite(y).all()
    y_ref = gold["y_ref"]
    err = float(np.max(np.abs(y[sample] - y_ref)) / np.max(np.abs(y_ref)))
    err2 = float(np.linalg.norm(y[sample] - y_ref) / np.linalg.norm(y_ref))
    print(f"sampled degrid max|dy|/max|y| {err:.2e}, norm {err2:.2e}", flush=True)
    assert err <= 1e-5


def test_sampled_grid(full):
    wl, uvw, x, ref, op, sample, gold = full
    yin = np.zeros(ref.m, dtype=np.complex128)
    yin[sample] = syn.random_vis(sample.size, seed=31)
    op.scratch.fill_(255)  # partial tiles and staging must all come from this call
    xa = op.grid(torch.from_numpy(yin)).cpu().numpy()
    assert np.isfinite(xa).all()
    rows, cols, xr = gold["rows"], gold["cols"], gold["x_ref"]
    err = float(np.max(np.abs(xa[rows, cols] - xr)) / np.max(np.abs(xr)))
    print(f"sampled grid max|dx|/max|x| {err:.2e} over {rows.size} pixels", flush=True)
    assert err <= 1e-5


def test_adjoint_identity_full_operator(full):
    # FP32 storage and accumulation over the whole operator
    wl, uvw, x, ref, op, sample, gold = full
    rel = adjoint_check.adjoint_gap(op, syn.random_image(wl.n, seed=41), seed=42)
    print(f"full adjoint identity {rel:.2e}", flush=True)
    assert rel <= 1e-6
