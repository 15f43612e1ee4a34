"""Edge and degenerate cases of the GPU operator, against the oracle.

One visibility; w exactly 0 (supports J, and -0.0 is not folded); every
visibility folded; w-stacks left empty by the assignment; visibilities many
grid widths away (taps wrap modulo G); supports wider than the grid (the
footprint wraps onto itself, so one visibility has several entries in one
tile); error paths (no visibilities, non-finite input, supports above
max_support, calls out of order); the w-plane mode with a single lattice
row and with non-default steps; a delta DDE kernel.  Bars as in the parity
tests: FP64 taps <= 1e-6 of the peak, operator ||d|| / || || <= 1e-5.
"""
import math

import numpy as np
import pytest
import torch

from oracle import dde, operator, presample, wkernel
from paper_1903_06555_amd import synthetic as syn
from paper_1903_06555_amd import wsp

pytestmark = pytest.mark.gpu


def check_operator(geom, uvw, ref, op, seed=0):
    x = syn.point_source_sky(geom.n, 6, "gaussian", seed=seed + 1, margin=3)
    y = op.degrid(torch.from_numpy(x)).cpu().numpy()
    y_ref = ref.forward(x)
    ey = float(np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref))
    yin = syn.random_vis(ref.m, seed=seed + 2)
    xa = op.grid(torch.from_numpy(yin)).cpu().numpy()
    xr = ref.adjoint(yin)
    ex = float(np.linalg.norm(xa - xr) / np.linalg.norm(xr))
    assert ey <= 1e-5 and ex <= 1e-5, (ey, ex)
    return ey, ex


def pair(geom, uvw, precision="fp64", **kw):
    """Oracle and GPU operators sharing one stack assignment."""
    n_stacks = kw.pop("n_stacks", 1)
    fold = kw.pop("fold", False)
    ref = operator.StackedOperator(geom, uvw, n_stacks=n_stacks, fold=fold, **kw)
    params = wsp.make_params(geom.n, geom.fov, n_stacks=n_stacks, fold=fold, precision=precision)
    op = wsp.Operator(params, uvw, labels=ref.labels, centres=ref.centres)
    return ref, op


G64 = wkernel.Geometry(n=64, fov=math.radians(10.0))


def test_one_visibility():
    uvw = np.array([[12.3, -7.9, 4.4]])
    ref, op = pair(G64, uvw)
    try:
        check_operator(G64, uvw, ref, op)
        K, u0, v0 = op.kernel(0)
        _, _, Kr = ref.kernel(0)
        assert np.max(np.abs(K - Kr)) <= 1e-6 * np.max(np.abs(Kr))
    finally:
        op.close()


def test_w_exactly_zero_and_negative_zero():
    uvw = syn.uniform_box_uvw(300, u_max=40.0, w_max=1.0, seed=101)
    uvw[:, 2] = 0.0
    uvw[::2, 2] = -0.0
    ref, op = pair(G64, uvw, fold=True)
    try:
        jp, folded = op.support()
        assert np.all(jp == G64.J) and not folded.any()
        check_operator(G64, uvw, ref, op, seed=102)
    finally:
        op.close()


def test_every_visibility_folded():
    uvw = syn.uniform_box_uvw(400, u_max=40.0, w_max=20.0, seed=103)
    uvw[:, 2] = -np.abs(uvw[:, 2]) - 0.5
    ref, op = pair(G64, uvw, fold=True, n_stacks=2)
    try:
        _, folded = op.support()
        assert folded.all()
        check_operator(G64, uvw, ref, op, seed=104)
    finally:
        op.close()


def test_empty_stacks():
    uvw = syn.uniform_box_uvw(300, u_max=40.0, w_max=20.0, seed=105)
    labels = np.zeros(300, dtype=np.int32)
    labels[::3] = 3
    centres = np.array([1.0, -50.0, 60.0, -2.0])  # stacks 1 and 2 have no members
    ref = operator.StackedOperator(G64, uvw, labels=labels, centres=centres)
    op = wsp.Operator(wsp.make_params(64, G64.fov, n_stacks=4, precision="fp64"), uvw,
                      labels=labels, centres=centres)
    try:
        check_operator(G64, uvw, ref, op, seed=106)
    finally:
        op.close()


def test_far_visibilities_wrap():
    # u, v up to ~5 grid widths away from the origin: taps wrap modulo G
    uvw = syn.uniform_box_uvw(300, u_max=40.0, w_max=20.0, seed=107)
    G_lambda = G64.grid_side * G64.du
    rng = np.random.default_rng(108)
    uvw[:, 0] += rng.integers(-5, 6, 300) * G_lambda + 0.37 * G_lambda
    uvw[:, 1] += rng.integers(-5, 6, 300) * G_lambda
    ref, op = pair(G64, uvw)
    try:
        check_operator(G64, uvw, ref, op, seed=109)
    finally:
        op.close()


def test_support_wider_than_grid():
    geom = wkernel.Geometry(n=64, fov=math.radians(25.0))
    uvw = syn.uniform_box_uvw(60, u_max=40.0, w_max=300.0, seed=110)
    ref, op = pair(geom, uvw)
    try:
        jp, _ = op.support()
        assert jp.max() > geom.grid_side  # the footprint wraps onto itself
        check_operator(geom, uvw, ref, op, seed=111)
    finally:
        op.close()


def test_error_paths():
    lib = wsp.load_library()
    params = wsp.make_params(64, G64.fov, precision="fp64")
    ctx = wsp.wsp_create(params)
    try:
        uvw = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
        with pytest.raises(wsp.WspError) as ei:
            wsp.wsp_set_uvw(ctx, uvw)
        assert ei.value.status == wsp.WSP_EINVAL
        bad = torch.tensor([[1.0, float("nan"), 0.0]], dtype=torch.float64, device="cuda")
        with pytest.raises(wsp.WspError) as ei:
            wsp.wsp_set_uvw(ctx, bad)
        assert ei.value.status == wsp.WSP_EINVAL
        # out of order: no visibilities yet
        assert lib.wsp_footprint(ctx, None, None, None) == wsp.WSP_ESTATE
        good = torch.tensor([[1.0, 2.0, 3.0]], dtype=torch.float64, device="cuda")
        wsp.wsp_set_uvw(ctx, good)
        img = torch.zeros((64, 64), dtype=torch.float64, device="cuda")
        vis = torch.zeros(1, dtype=torch.complex128, device="cuda")
        with pytest.raises(wsp.WspError) as ei:
            wsp.wsp_degrid(ctx, img, vis)  # not bound, not built
        assert ei.value.status == wsp.WSP_ESTATE
    finally:
        wsp.wsp_destroy(ctx)
    # supports above max_support (one stack centred at w = 100: |w_eff| = 100, J_p = 14)
    small = wsp.make_params(64, G64.fov, precision="fp64", max_support=8)
    with pytest.raises(wsp.WspError) as ei:
        wsp.Operator(small, np.array([[1.0, 2.0, 0.0], [3.0, 4.0, 200.0]]))
    assert ei.value.status == wsp.WSP_ESUPPORT


def test_planes_single_row_lattice():
    # every |w_eff| below dw: one pair row
    geom = wkernel.Geometry(n=64, fov=math.radians(25.0))
    uvw = syn.uniform_box_uvw(500, u_max=40.0, w_max=0.03, seed=112)
    ps = presample.PlaneSampler(geom)
    labels = np.zeros(500, dtype=np.int32)
    centres = np.array([0.0])
    ref = operator.StackedOperator(geom, uvw, labels=labels, centres=centres,
                                   kernel_fn=ps.visibility_kernel)
    op = wsp.Operator(wsp.make_params(64, geom.fov, kernels="planes"), uvw, labels=labels,
                      centres=centres)
    try:
        assert op.footprint["kernel_bytes"] < 16 * 64 * 8  # one short row
        check_operator(geom, uvw, ref, op, seed=113)
    finally:
        op.close()


def test_planes_custom_steps():
    geom = wkernel.Geometry(n=64, fov=math.radians(25.0))
    dq, dw = 1.0 / 32.0, 1.0 / 8.0
    uvw = syn.uniform_box_uvw(600, u_max=40.0, w_max=25.0, seed=114)
    ps = presample.PlaneSampler(geom, dq, dw)
    ref0 = operator.StackedOperator(geom, uvw, n_stacks=2, fold=True)
    ref = operator.StackedOperator(geom, uvw, labels=ref0.labels, centres=ref0.centres, fold=True,
                                   kernel_fn=ps.visibility_kernel)
    params = wsp.make_params(64, geom.fov, n_stacks=2, fold=True, kernels="planes", plane_dq=dq,
                             plane_dw=dw)
    op = wsp.Operator(params, uvw, labels=ref.labels, centres=ref.centres)
    try:
        check_operator(geom, uvw, ref, op, seed=115)
    finally:
        op.close()


def test_delta_dde_is_the_plain_operator():
    uvw = syn.uniform_box_uvw(400, u_max=40.0, w_max=20.0, seed=116)
    m = uvw.shape[0]
    d = np.zeros((m, 3), dtype=complex)
    d[:, 1] = 1.0
    ref = operator.StackedOperator(G64, uvw, n_stacks=2, fold=True)
    a = wsp.Operator(wsp.make_params(64, G64.fov, n_stacks=2, fold=True, precision="fp64", dde_support=3),
                     uvw, labels=ref.labels, centres=ref.centres, build=False)
    try:
        a.set_dde(d, d)
        a.build()
        check_operator(G64, uvw,
                       operator.StackedOperator(G64, uvw, labels=ref.labels, centres=ref.centres, fold=True,
                                                kernel_fn=dde.DDEKernels(d, d), extra_support=2),
                       a, seed=117)
        x = torch.from_numpy(syn.point_source_sky(64, 6, "gaussian", seed=118, margin=3))
        y = a.degrid(x).cpu().numpy()
        y_plain = ref.forward(x.numpy())
        assert np.linalg.norm(y - y_plain) <= 1e-5 * np.linalg.norm(y_plain)
    finally:
        a.close()


def test_forced_quadrature_cap_warns_and_completes():
    """A panel cap far below what wide w needs: the build stops refining, returns
    WSP_WARN_QUAD_MAXEVAL with the count of capped visibilities, and still exits
    normally with every tap and output finite."""
    uvw = np.array([[10.0, 5.0, 400.0], [3.0, -2.0, 350.0], [-7.0, 4.0, -300.0], [1.0, 1.0, 0.0]])
    params = wsp.make_params(256, math.radians(25.0), quad_max_panels=8, max_support=512)
    op = wsp.Operator(params, uvw, build=False)
    with pytest.warns(UserWarning, match="quadrature tolerance"):
        status = op.build()
    assert status == wsp.WSP_WARN_QUAD_MAXEVAL
    panels, capped = op.quad_stats()
    print(f"capped {capped} of {op.m}, panels {panels}", flush=True)
    assert 3 <= capped <= op.m and panels <= 8 * op.m
    for p in range(op.m):
        assert np.isfinite(op.kernel(p)[0]).all()
    y = op.degrid(torch.from_numpy(syn.point_source_sky(256, 10, "exp", 3))).cpu().numpy()
    assert np.isfinite(y).all()
    # the default cap meets the tolerance on the same visibilities
    full = wsp.Operator(wsp.make_params(256, math.radians(25.0), max_support=512), uvw)
    assert full.build_status == wsp.WSP_OK and full.quad_stats()[1] == 0
    op.close()
    full.close()
