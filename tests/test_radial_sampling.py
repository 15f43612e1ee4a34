"""The radial-sample construction is numerically sound (CPU, oracle only).

K_p depends on a tap only through its distance q and is band-limited, so the
GPU builder evaluates the Eq. (6) quadrature at q = s h (h = 1/8 cell on the
FP64 path, 1/6 on the FP32 path) and interpolates each tap from the 10
samples around it.  This checks, with the FP64 oracle's kernel alone, that
such an interpolant reproduces direct evaluation far below the 1e-6 kernel
tolerance (below 1e-8 at h = 1/8, below 1e-7 at h = 1/6), at w = 0 and at
large |w - wbar| of the 1024^2, 25 deg workload, and that a coarser step
would not.
"""
import math

import numpy as np
import pytest

from oracle import wkernel

POINTS = 10


def interpolate(samples, q, step, points):
    """Equispaced Lagrange interpolation of K(|s| step) at q (K is even in q)."""
    x = q / step
    s0 = int(math.floor(x)) - (points // 2 - 1)
    nodes = np.arange(s0, s0 + points)
    vals = samples[np.abs(nodes)]
    out = 0.0
    for k in range(points):
        lk = 1.0
        for j in range(points):
            if j != k:
                lk *= (x - nodes[j]) / (nodes[k] - nodes[j])
        out = out + lk * vals[k]
    return out


@pytest.mark.parametrize("weff", [0.0, -250.0])
@pytest.mark.parametrize("step,bound", [(1.0 / 8.0, 1e-8), (1.0 / 6.0, 1e-7)])
def test_interpolated_kernel_matches_direct(weff, step, bound):
    geom = wkernel.Geometry(n=1024, fov=math.radians(25.0))
    jp = int(wkernel.support(weff, geom))
    qmax = (jp / 2 + 1) * math.sqrt(2.0)  # beyond the corner tap of a J_p x J_p block
    rng = np.random.default_rng(3)
    q = rng.uniform(0.0, qmax, 120)
    direct = wkernel.wkernel(q, weff, geom)
    n_samples = int(math.floor(qmax / step)) + POINTS // 2 + 1
    samples = wkernel.wkernel(np.arange(n_samples) * step, weff, geom)
    peak = float(np.max(np.abs(samples)))
    interp = np.array([interpolate(samples, qq, step, POINTS) for qq in q])
    err = float(np.max(np.abs(interp - direct))) / peak
    assert err < bound, err
    # a step twice as coarse misses the bar: the check has teeth
    coarse = wkernel.wkernel(np.arange(n_samples // 2 + POINTS) * (2 * step), weff, geom)
    interp_c = np.array([interpolate(coarse, qq, 2 * step, POINTS) for qq in q[:40]])
    err_c = float(np.max(np.abs(interp_c - direct[:40]))) / peak
    assert err_c > 10 * bound, err_c
