"""Model error of the w-stacking w-projection operator against Eq. (1).

Parity tests compare the GPU with the oracle's version of the same
approximation (Eqs. (4)-(7)); this test measures the approximation itself:
the GPU's degridded visibilities of the workload's point-source sky against
the measurement equation evaluated directly (oracle.dft.measure, FP64), on
2000 visibilities stratified by |w - wbar| (uniform quantiles, the largest
included), for support scales f = 1, 2, 4 of the w-kernel support rule
J_p = J + 2 ceil(|w - wbar| s f).

Each visibility's output depends only on its own kernel and its stack's
grid, so the sample is applied as an operator of its own with the full
set's stack assignment and centres (wsp_set_stacks).

What is checked: the error does not grow with f (a wider support keeps
more of each w-projection kernel), and at f = 4 it is within twice the
Kaiser-Bessel gridding's own aliasing floor (J = 4, alpha = 2), measured as
the error of the same visibilities with w = 0 (no w-term at all).  The
figures are printed and reported with the design notes.
"""
import math

import numpy as np
import pytest
import torch

from oracle import dft
from paper_1903_06555_amd import synthetic as syn
from paper_1903_06555_amd import wsp

pytestmark = pytest.mark.gpu

WORKLOADS = ["mwa_1024_single_stack", "mwa_4096_16_stacks"]
SCALES = [1.0, 2.0, 4.0]
N_SAMPLE = 2000


def _sample(uvw, labels, centres, fold):
    # uniform quantiles of the distance |w_eff - wbar| in wavelengths (Eq. (8)
    # folds w onto |w|)
    w_eff = np.abs(uvw[:, 2]) if fold else uvw[:, 2]
    dist = np.abs(w_eff - centres[labels])
    order = np.argsort(dist, kind="stable")
    pick = np.unique(np.round(np.linspace(0, order.size - 1, N_SAMPLE)).astype(np.int64))
    return np.sort(order[pick])


def _rel(y, y_ref):
    return float(np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref))


@pytest.fixture(scope="module", params=WORKLOADS)
def workload(request):
    wl = syn.WORKLOADS[request.param]
    uvw = syn.workload_uvw(wl)
    fov = math.radians(wl.fov_deg)
    params = wsp.make_params(wl.n, fov, n_stacks=wl.n_stacks, fold=wl.fold, precision=wl.precision)
    op = wsp.Operator(params, uvw, build=False)
    labels, centres, _ = op.stacks()
    op.close()
    torch.cuda.empty_cache()
    sample = _sample(uvw, labels, centres, wl.fold)
    sky = syn.workload_sky(wl)
    return wl, fov, uvw[sample], labels[sample], centres, sky


def _degrid(wl, fov, uvw, labels, centres, sky, f):
    params = wsp.make_params(wl.n, fov, n_stacks=wl.n_stacks, fold=wl.fold, precision=wl.precision,
                             support_scale=f, max_support=8192)
    op = wsp.Operator(params, uvw, labels=labels, centres=centres)
    try:
        assert op.build_status == wsp.WSP_OK
        jp, _ = op.support()
        y = op.degrid(torch.from_numpy(sky)).cpu().numpy().astype(np.complex128)
    finally:
        op.close()
    return y, jp


def test_model_error_against_measurement_equation(workload):
    wl, fov, uvw, labels, centres, sky = workload
    y_true = dft.measure(sky, uvw, fov)
    errs, mean_jp = {}, {}
    for f in SCALES:
        y, jp = _degrid(wl, fov, uvw, labels, centres, sky, f)
        errs[f] = _rel(y, y_true)
        mean_jp[f] = float(np.mean(jp))
    # the gridding floor: the same visibilities with w = 0, every stack centre at 0
    flat = uvw.copy()
    flat[:, 2] = 0.0
    y0, _ = _degrid(wl, fov, flat, labels, np.zeros_like(centres), sky, 1.0)
    floor = _rel(y0, dft.measure(sky, flat, fov))
    print(f"{wl.name}: model error vs Eq. (1) on {uvw.shape[0]} visibilities: " +
          ", ".join(f"f={f:g}: {errs[f]:.3e} (mean J_p {mean_jp[f]:.1f})" for f in SCALES) +
          f"; gridding floor (w = 0) {floor:.3e}", flush=True)
    assert errs[2.0] <= errs[1.0] * 1.01
    assert errs[4.0] <= errs[2.0] * 1.01
    assert errs[4.0] <= 2.0 * floor
    assert floor < 1e-2
