"""GPU parity of the DDE convolution of the kernels (Sec. 5.2, Eq. (11)).

The GPU builds each visibility's Eq. (6) taps on the inner J_p x J_p block of
a J_p + J_D - 1 support and convolves them in place with the visibility's
separable D (two 1-D passes); the oracle convolves its FP64 taps with the
outer product D (oracle/dde.py).  Bars: taps max|dK'| / max|K'| <= 1e-6 (the
quadrature tolerance; D is O(1)), degrid and grid ||d|| / || || <= 1e-5.
A unit-shift D must turn the GPU operator into the GPU operator at u + du
(Fourier shift theorem).  A folded full-size workload (2048^2, 5e6
visibilities, 8 stacks, J_D = 3) is checked on a stratified sample.
"""
import math

import numpy as np
import pytest
import torch

from oracle import dde, operator, stacking, wkernel
from paper_1903_06555_amd import synthetic as syn
from paper_1903_06555_amd import wsp

pytestmark = pytest.mark.gpu

N, FOV, JD = 64, math.radians(10.0), 5


def random_dde(m, jd, seed):
    rng = np.random.default_rng(seed)
    mk = lambda: (rng.normal(size=(m, jd)) + 1j * rng.normal(size=(m, jd))) / jd
    return mk(), mk()


@pytest.fixture(scope="module", params=["fp64", "fp32_fp64phase"])
def tiny(request):
    geom = wkernel.Geometry(n=N, fov=FOV)
    uvw = syn.uniform_box_uvw(1500, u_max=40.0, w_max=20.0, seed=91)
    wts = np.random.default_rng(92).uniform(0.5, 1.5, uvw.shape[0])
    plain = operator.StackedOperator(geom, uvw, n_stacks=3, fold=True)
    du, dv = random_dde(plain.m, JD, 93)
    ref = operator.StackedOperator(geom, uvw, weights=wts, labels=plain.labels, centres=plain.centres,
                                   fold=True, kernel_fn=dde.DDEKernels(du, dv), extra_support=JD - 1)
    params = wsp.make_params(N, FOV, n_stacks=3, fold=True, precision=request.param, dde_support=JD)
    op = wsp.Operator(params, uvw, weights=wts, labels=ref.labels, centres=ref.centres, build=False)
    with pytest.raises(wsp.WspError) as ei:
        op.build()  # the DDE kernels are not set yet
    assert ei.value.status == wsp.WSP_ESTATE
    op.set_dde(du, dv)
    assert op.build() == 0
    yield request.param, ref, op
    op.close()


def test_tiny_supports(tiny):
    precision, ref, op = tiny
    jp, _ = op.support()
    assert np.array_equal(jp, ref.jp)
    assert np.array_equal(jp, dde.support(ref.w_eff, ref.geom, JD))


def test_tiny_every_tap(tiny):
    precision, ref, op = tiny
    worst = 0.0
    for p in range(ref.m):
        K, u0, v0 = op.kernel(p)
        ru0, rv0, Kr = ref.kernel(p)
        assert (u0, v0) == (ru0, rv0)
        err = float(np.max(np.abs(K - Kr)) / np.max(np.abs(Kr)))
        worst = max(worst, err)
    print(f"{precision}: DDE taps max |dK'| / max|K'| = {worst:.2e}", flush=True)
    assert worst <= 1e-6


def test_tiny_operator(tiny):
    precision, ref, op = tiny
    x = syn.point_source_sky(N, 12, "gaussian", seed=94, margin=4)
    y = op.degrid(torch.from_numpy(x)).cpu().numpy()
    y_ref = ref.forward(x)
    ey = float(np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref))
    yin = syn.random_vis(ref.m, seed=95)
    xa = op.grid(torch.from_numpy(yin)).cpu().numpy()
    xr = ref.adjoint(yin)
    ex = float(np.linalg.norm(xa - xr) / np.linalg.norm(xr))
    print(f"{precision}: DDE degrid {ey:.2e} grid {ex:.2e}", flush=True)
    assert ey <= 1e-5 and ex <= 1e-5


def test_unit_shift_equals_shifted_uv():
    geom = wkernel.Geometry(n=N, fov=FOV)
    uvw = syn.uniform_box_uvw(800, u_max=40.0, w_max=20.0, seed=96)
    m = uvw.shape[0]
    du = np.zeros((m, 3), dtype=complex)
    dv = np.zeros((m, 3), dtype=complex)
    du[:, 2] = 1.0
    dv[:, 1] = 1.0
    labels = np.zeros(m, dtype=np.int32)
    centres = np.array([0.0])
    a = wsp.Operator(wsp.make_params(N, FOV, precision="fp64", dde_support=3), uvw, labels=labels,
                     centres=centres, build=False)
    uvw_s = uvw.copy()
    uvw_s[:, 0] += geom.du
    b = wsp.Operator(wsp.make_params(N, FOV, precision="fp64"), uvw_s, labels=labels, centres=centres)
    try:
        a.set_dde(du, dv)
        a.build()
        x = torch.from_numpy(syn.point_source_sky(N, 8, "gaussian", seed=97, margin=4))
        ya, yb = a.degrid(x).cpu().numpy(), b.degrid(x).cpu().numpy()
        err = float(np.linalg.norm(ya - yb) / np.linalg.norm(yb))
        print(f"unit-shift DDE vs shifted uv: {err:.2e}", flush=True)
        assert err <= 1e-5
    finally:
        a.close()
        b.close()


def test_dde_lds_limit():
    # 15-wide D on supports near 300 taps does not fit the convolution's LDS ring
    uvw = syn.uniform_box_uvw(50, u_max=40.0, w_max=500.0, seed=98)
    params = wsp.make_params(1024, math.radians(25.0), precision="fp64", dde_support=15)
    with pytest.raises(wsp.WspError) as ei:
        wsp.Operator(params, uvw, build=False)
    assert ei.value.status == wsp.WSP_ESUPPORT


def test_fullsize_sampled_dde():
    wl = syn.WORKLOADS["mwa_2048_8_stacks"]
    jd = 3
    uvw = syn.workload_uvw(wl)
    geom = wkernel.Geometry(n=wl.n, fov=math.radians(wl.fov_deg))
    folded, _ = stacking.fold(uvw)
    labels, centres, _ = stacking.kmeans_w(folded[:, 2], wl.n_stacks, 1e-3, 100)
    du, dv = random_dde(uvw.shape[0], jd, 99)
    ref = operator.StackedOperator(geom, uvw, labels=labels, centres=centres, fold=True,
                                   kernel_fn=dde.DDEKernels(du, dv), extra_support=jd - 1)
    params = wsp.make_params(wl.n, geom.fov, n_stacks=wl.n_stacks, fold=True, precision=wl.precision,
                             dde_support=jd)
    op = wsp.Operator(params, uvw, labels=labels, centres=centres, build=False)
    try:
        op.set_dde(du, dv)
        op.build()
        order = np.argsort(ref.jp, kind="stable")
        sample = np.unique(order[(np.array([0.01, 0.3, 0.6, 0.9, 0.99, 1.0]) * (ref.m - 1)).astype(int)])
        for p in sample:
            K, _, _ = op.kernel(int(p))
            _, _, Kr = ref.kernel(int(p))
            assert np.max(np.abs(K - Kr)) <= 1e-6 * np.max(np.abs(Kr)), p
        x = syn.workload_sky(wl)
        op.scratch.fill_(255)
        y = op.degrid(torch.from_numpy(x)).cpu().numpy()
        y_ref = ref.forward(x, subset=sample)[sample]
        err = float(np.linalg.norm(y[sample] - y_ref) / np.linalg.norm(y_ref))
        print(f"{wl.name} DDE J_D {jd}: sampled degrid rel err {err:.2e}", flush=True)
        assert err <= 1e-5
    finally:
        op.close()


def test_dde_build_in_parts_and_after_restack():
    """A part-wise build gives the same taps; DDE kernels survive wsp_set_stacks."""
    geom = wkernel.Geometry(n=N, fov=FOV)
    uvw = syn.uniform_box_uvw(900, u_max=40.0, w_max=20.0, seed=120)
    du, dv = random_dde(uvw.shape[0], 3, 121)
    params = wsp.make_params(N, FOV, n_stacks=2, fold=True, precision="fp64", dde_support=3)
    a = wsp.Operator(params, uvw, build=False)
    b = wsp.Operator(params, uvw, build=False)
    try:
        labels, centres, _ = a.stacks()
        b.set_stacks(labels, centres)
        a.set_dde(du, dv)
        b.set_dde(du, dv)
        a.build()
        seen = []
        b.build(part=250, progress=lambda d, n: seen.append(d))
        assert seen == [250, 500, 750, 900]
        x = torch.from_numpy(syn.point_source_sky(N, 8, "gaussian", seed=122, margin=4))
        assert torch.equal(a.degrid(x), b.degrid(x))
        # re-plan with another assignment: the DDE kernels are kept, the taps rebuilt
        other = np.zeros(uvw.shape[0], dtype=np.int32)
        b.set_stacks(other, np.array([0.0, 5.0]))
        b.build()
        ref = operator.StackedOperator(geom, uvw, labels=other, centres=np.array([0.0, 5.0]), fold=True,
                                       kernel_fn=dde.DDEKernels(du, dv), extra_support=2)
        y = b.degrid(x).cpu().numpy()
        y_ref = ref.forward(x.numpy())
        assert np.linalg.norm(y - y_ref) <= 1e-5 * np.linalg.norm(y_ref)
    finally:
        a.close()
        b.close()
