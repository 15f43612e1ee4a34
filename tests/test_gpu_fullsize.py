"""GPU parity at the benchmark's full size, in the benchmark's launch configuration.

Workload: 1024^2 image, 25 deg, 1e6 MWA-like visibilities, one w-stack,
FP32 data with FP64 phases (mean J_p 87, max 282, 88 GB of taps).  The
oracle cannot evaluate a million kernels, so it checks a stratified sample
of visibilities one by one (kernel taps, degridded values, and the gridded
image of a visibility vector that is non-zero only on the sample); the
adjoint identity is checked on the whole operator.
"""
import math

import numpy as np
import pytest
import torch

from oracle import operator, wkernel
from paper_1903_06555_amd import synthetic as syn
from paper_1903_06555_amd import wsp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    wl = syn.WORKLOADS["mwa_1024_single_stack"]
    uvw = syn.workload_uvw(wl)
    x = syn.workload_sky(wl)
    geom = wkernel.Geometry(n=wl.n, fov=math.radians(wl.fov_deg))
    ref = operator.StackedOperator(geom, uvw, n_stacks=1)
    params = wsp.make_params(wl.n, geom.fov, n_stacks=1, precision=wl.precision)
    op = wsp.Operator(params, uvw, labels=ref.labels, centres=ref.centres, build=False)
    op.build(part=200_000, progress=lambda d, n: print(f"built {d}/{n}", flush=True))
    order = np.argsort(ref.jp, kind="stable")
    qs = [0.02, 0.3, 0.6, 0.9, 0.99]
    sample = np.unique(order[(np.array(qs) * (ref.m - 1)).astype(int)])
    print("sample J_p:", ref.jp[sample].tolist(), flush=True)
    yield wl, uvw, x, ref, op, sample
    op.close()


def test_supports_bit_exact(full):
    wl, uvw, x, ref, op, sample = full
    jp, folded = op.support()
    assert np.array_equal(jp, ref.jp)
    assert not folded.any()


def test_sampled_kernels(full):
    wl, uvw, x, ref, op, sample = full
    for p in sample:
        K, u0, v0 = op.kernel(int(p))
        ru0, rv0, Kr = ref.kernel(int(p))
        assert (u0, v0) == (ru0, rv0)
        err = float(np.max(np.abs(K - Kr)) / np.max(np.abs(Kr)))
        print(f"vis {p} J_p {K.shape[0]}: max|dK|/max|K| = {err:.2e}", flush=True)
        assert err <= 1e-6


def test_sampled_degrid(full):
    wl, uvw, x, ref, op, sample = full
    # every per-entry partial must come from this call: poison the scratch
    op.scratch.fill_(255)
    y = op.degrid(torch.from_numpy(x)).cpu().numpy()
    assert np.isfinite(y).all()
    y_ref = ref.forward(x, subset=sample)[sample]
    err = float(np.linalg.norm(y[sample] - y_ref) / np.linalg.norm(y_ref))
    print(f"sampled degrid rel err {err:.2e}", flush=True)
    assert err <= 1e-5


def test_sampled_grid(full):
    wl, uvw, x, ref, op, sample = full
    yin = np.zeros(ref.m, dtype=np.complex128)
    yin[sample] = syn.random_vis(sample.size, seed=31)
    op.scratch.fill_(255)  # partial tiles and staging must all come from this call
    xa = op.grid(torch.from_numpy(yin)).cpu().numpy()
    assert np.isfinite(xa).all()
    xr = ref.adjoint(yin, subset=sample)
    err = float(np.linalg.norm(xa - xr) / np.linalg.norm(xr))
    print(f"sampled grid rel err {err:.2e}", flush=True)
    assert err <= 1e-5


def test_adjoint_identity_full_operator(full):
    # FP32 storage and accumulation: the identity holds to single precision
    wl, uvw, x, ref, op, sample = full
    xr = torch.from_numpy(syn.random_image(wl.n, seed=41))
    yr = torch.from_numpy(syn.random_vis(ref.m, seed=42))
    Phx = op.degrid(xr).cpu().numpy().astype(np.complex128)
    Phty = op.grid(yr).cpu().numpy().astype(np.float64)
    lhs = float(np.real(np.vdot(Phx, yr.numpy())))
    rhs = float(np.sum(xr.numpy() * Phty))
    rel = abs(lhs - rhs) / abs(lhs)
    print(f"full adjoint identity {rel:.2e}", flush=True)
    assert rel <= 1e-4
