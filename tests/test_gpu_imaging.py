"""Imaging loop on the GPU operator: power method, FISTA and ADMM.

On a 32^2 problem the GPU (all-FP64 path) and the oracle drive the same
loop; the operators agree to the kernels' quadrature tolerance, so ||Phi||^2
and the FISTA iterates agree to ~1e-6.  On the 2048^2, 5e6-visibility,
8-stack workload the FP32 loop follows the all-FP64 loop iterate by iterate.
"""
import math
import time

import numpy as np
import pytest
import torch

from oracle import operator, wkernel
from paper_1903_06555_amd import imaging, wsp
from paper_1903_06555_amd import synthetic as syn

pytestmark = pytest.mark.gpu


class OracleOp:
    def __init__(self, n, fov_deg, uvw, labels, centres):
        self.ref = operator.StackedOperator(wkernel.Geometry(n=n, fov=math.radians(fov_deg)), uvw,
                                            labels=labels, centres=centres)
        self.n = n
        self.device = torch.device("cpu")
        self.real_dtype = torch.float64

    def degrid(self, x):
        return torch.from_numpy(self.ref.forward(x.cpu().numpy()))

    def grid(self, y):
        return torch.from_numpy(self.ref.adjoint(y.cpu().numpy()))


def test_power_and_fista_match_oracle():
    n, fov = 32, 10.0
    uvw = syn.uniform_box_uvw(600, u_max=25.0, w_max=15.0, seed=23)
    labels = np.zeros(len(uvw), dtype=np.int32)
    centres = np.array([0.0])
    ora = OracleOp(n, fov, uvw, labels, centres)
    params = wsp.make_params(n, math.radians(fov), precision="fp64")
    gpu = wsp.Operator(params, uvw, labels=labels, centres=centres)
    try:
        sky = syn.point_source_sky(n, 6, "exp", seed=24, margin=4)
        y_cpu = ora.degrid(torch.from_numpy(sky))
        L_o = imaging.power_norm2(ora, n_iter=60)
        L_g = imaging.power_norm2(gpu, n_iter=60)
        assert abs(L_g - L_o) <= 1e-6 * L_o, (L_g, L_o)
        lam = 0.02 * float(torch.max(torch.abs(ora.grid(y_cpu))))
        r_o = imaging.fista_l1(ora, y_cpu, lam, n_iter=60, norm2=L_o, track=False)
        r_g = imaging.fista_l1(gpu, y_cpu.cuda(), lam, n_iter=60, norm2=L_o, track=False)
        x_o, x_g = r_o.x.numpy(), r_g.x.cpu().numpy()
        err = float(np.linalg.norm(x_g - x_o) / np.linalg.norm(x_o))
        print(f"||Phi||^2 gpu {L_g:.9e} oracle {L_o:.9e}; FISTA iterate rel diff {err:.2e}", flush=True)
        assert err <= 1e-5
    finally:
        gpu.close()


def test_admm_matches_oracle():
    n, fov = 32, 10.0
    uvw = syn.uniform_box_uvw(600, u_max=25.0, w_max=15.0, seed=25)
    labels = np.zeros(len(uvw), dtype=np.int32)
    centres = np.array([0.0])
    ora = OracleOp(n, fov, uvw, labels, centres)
    gpu = wsp.Operator(wsp.make_params(n, math.radians(fov), precision="fp64"), uvw, labels=labels,
                       centres=centres)
    try:
        sky = syn.point_source_sky(n, 6, "exp", seed=26, margin=4)
        y = ora.degrid(torch.from_numpy(sky))
        L = imaging.power_norm2(ora, n_iter=60)
        eps = 0.05 * float(torch.linalg.vector_norm(y))
        mu = 0.01 * float(torch.max(torch.abs(ora.grid(y))))
        r_o = imaging.admm_l1_ball(ora, y, eps, mu, n_iter=80, norm2=L)
        r_g = imaging.admm_l1_ball(gpu, y.cuda(), eps, mu, n_iter=80, norm2=L)
        x_o, x_g = r_o.x.numpy(), r_g.x.cpu().numpy()
        err = float(np.linalg.norm(x_g - x_o) / np.linalg.norm(x_o))
        print(f"ADMM (Eq. 10, eps-ball) GPU vs oracle iterate rel diff {err:.2e}, residual "
              f"{r_g.residual[-1]:.4e} (eps {eps:.4e})", flush=True)
        assert err <= 1e-5
        assert abs(r_g.residual[-1] - r_o.residual[-1]) <= 1e-5 * r_o.residual[-1]
    finally:
        gpu.close()


def test_fista_8_stacks_fp32_follows_fp64():
    """FISTA on the 2048^2, 5e6-visibility, 8-stack workload: the FP32 loop
    follows the all-FP64 loop (whose operator is pinned to the oracle by the
    parity tests) iterate by iterate, to FP32 accuracy, and keeps x >= 0."""
    wl = syn.WORKLOADS["mwa_2048_8_stacks"]
    uvw = syn.workload_uvw(wl)
    runs = {}
    labels = centres = None
    for precision in ("fp64", "fp32_fp64phase"):
        params = wsp.make_params(wl.n, math.radians(wl.fov_deg), n_stacks=wl.n_stacks, fold=wl.fold,
                                 precision=precision)
        op = wsp.Operator(params, uvw, labels=labels, centres=centres)
        if labels is None:
            labels, centres, _ = op.stacks()
        try:
            sky = torch.from_numpy(syn.workload_sky(wl)).cuda().to(op.real_dtype)
            y = op.degrid(sky)
            if precision == "fp64":
                L = imaging.power_norm2(op, n_iter=20)
                lam = 1e-3 * float(torch.max(torch.abs(op.grid(y))))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = imaging.fista_l1(op, y, lam, n_iter=8, norm2=L)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / 8
            runs[precision] = (res.x.double().cpu().numpy(), res.objective)
            print(f"{precision} FISTA: {dt * 1e3:.1f} ms per iteration (with objective), objective "
                  f"{res.objective[0]:.6e} -> {res.objective[-1]:.6e}", flush=True)
            assert float(res.x.min()) >= 0.0
        finally:
            op.close()
    (x64, o64), (x32, o32) = runs["fp64"], runs["fp32_fp64phase"]
    err = float(np.linalg.norm(x32 - x64) / np.linalg.norm(x64))
    print(f"FP32 vs FP64 iterate after 8 iterations: {err:.2e}", flush=True)
    assert err <= 1e-4
    assert max(abs(a - b) / abs(b) for a, b in zip(o32, o64)) <= 1e-4
