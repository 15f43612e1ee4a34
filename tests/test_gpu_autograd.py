"""Differentiable operator: degrid forward, gridding backward (GPU)."""
import math

import numpy as np
import pytest
import torch

from oracle import operator, wkernel
from paper_1903_06555_amd import synthetic as syn
from paper_1903_06555_amd import wsp
from paper_1903_06555_amd.autograd import degrid, power_norm2

pytestmark = pytest.mark.gpu


def _small_op(precision):
    uvw = syn.uniform_box_uvw(300, u_max=50.0, w_max=30.0, seed=51)
    wts = syn.random_weights(300, seed=52)
    params = wsp.make_params(32, math.radians(10.0), n_stacks=2, fold=True, precision=precision)
    return wsp.Operator(params, uvw, weights=wts)


def test_gradcheck_fp64():
    op = _small_op("fp64")
    x = torch.from_numpy(syn.random_image(32, seed=53)).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda z: degrid(z, op), (x,), eps=1e-6, atol=1e-8,
                                    rtol=1e-6, fast_mode=True)
    op.close()


def test_backward_is_gridding():
    op = _small_op("fp32_fp64phase")
    x = torch.from_numpy(syn.random_image(32, seed=54)).float().cuda().requires_grad_(True)
    d = torch.from_numpy(syn.random_vis(op.m, seed=55)).to(torch.complex64).cuda()
    y = degrid(x, op)
    loss = 0.5 * torch.sum(torch.abs(y - d) ** 2)
    loss.backward()
    expect = op.grid((op.degrid(x.detach()) - d))
    assert torch.allclose(x.grad, expect, rtol=1e-5, atol=1e-5 * float(expect.abs().max()))
    op.close()


@pytest.fixture(scope="module")
def lsq():
    """Least-squares problem at the 2048^2 / 5e6 visibility / 8 stack shape."""
    wl = syn.WORKLOADS["mwa_2048_8_stacks"]
    uvw = syn.workload_uvw(wl)
    fov = math.radians(wl.fov_deg)
    p64 = wsp.make_params(wl.n, fov, n_stacks=wl.n_stacks, fold=True, precision="fp64")
    op64 = wsp.Operator(p64, uvw, build=False)
    op64.build(part=1_000_000, progress=lambda a, b: print(f"fp64 built {a}/{b}", flush=True))
    labels, centres, _ = op64.stacks()
    p32 = wsp.make_params(wl.n, fov, n_stacks=wl.n_stacks, fold=True, precision="fp32_fp64phase")
    op32 = wsp.Operator(p32, uvw, labels=labels, centres=centres, build=False)
    op32.build(part=1_000_000, progress=lambda a, b: print(f"fp32 built {a}/{b}", flush=True))
    x_true = torch.from_numpy(syn.workload_sky(wl)).cuda()
    d = op64.degrid(x_true)
    yield wl, op64, op32, x_true, d
    op64.close()
    op32.close()


def test_adjoint_identity_fp64_full(lsq):
    wl, op64, op32, x_true, d = lsq
    x = torch.from_numpy(syn.random_image(wl.n, seed=61)).cuda()
    y = torch.from_numpy(syn.random_vis(op64.m, seed=62)).cuda()
    lhs = float(torch.real(torch.vdot(op64.degrid(x), y)))
    rhs = float(torch.sum(x * op64.grid(y)))
    print(f"fp64 adjoint identity at 2048^2 / 5e6: {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_least_squares_gradient_step(lsq):
    wl, op64, op32, x_true, d = lsq
    eta = 1.0 / power_norm2(op32, n_iter=15)
    x0 = torch.zeros(wl.n, wl.n, dtype=torch.float32, device="cuda", requires_grad=True)
    d32 = d.to(torch.complex64)

    def loss(z):
        return 0.5 * torch.sum(torch.abs(degrid(z, op32) - d32) ** 2)

    l0 = loss(x0)
    l0.backward()
    with torch.no_grad():
        x1 = x0 - eta * x0.grad
    l1 = loss(x1)
    print(f"eta {eta:.3e}: loss {float(l0):.6e} -> {float(l1):.6e}")
    assert float(l1) < float(l0)
    # the step moves toward the true sky: correlation with x_true is positive
    assert float(torch.sum(x1 * x_true.float())) > 0


def test_finite_difference_along_direction_fp64(lsq):
    wl, op64, op32, x_true, d = lsq
    x = (0.5 * x_true).clone().requires_grad_(True)
    loss = lambda z: 0.5 * torch.sum(torch.abs(degrid(z, op64) - d) ** 2)
    l = loss(x)
    l.backward()
    direc = torch.from_numpy(syn.random_image(wl.n, seed=63)).cuda()
    analytic = float(torch.sum(x.grad * direc))
    eps = 1e-3
    with torch.no_grad():
        fd = (float(loss(x + eps * direc)) - float(loss(x - eps * direc))) / (2 * eps)
    print(f"directional derivative: analytic {analytic:.12e} fd {fd:.12e}")
    # the loss is quadratic, so the central difference is exact up to rounding
    assert abs(analytic - fd) <= 1e-6 * abs(analytic)
