"""Served operator: mixed request streams give the same results as requests alone."""
import math

import numpy as np
import pytest
import torch

from paper_1903_06555_amd import synthetic as syn
from paper_1903_06555_amd import wsp
from paper_1903_06555_amd.serving import Server, job_footprint_bytes

pytestmark = pytest.mark.gpu

JOBS = [  # (name, n, fov_deg, m, stacks, fold, precision)
    ("a", 64, 10.0, 3000, 1, False, "fp32_fp64phase"),
    ("b", 128, 25.0, 2000, 3, True, "fp32_fp64phase"),
    ("c", 64, 10.0, 1500, 2, True, "fp64"),
    ("d", 256, 25.0, 4000, 4, True, "fp32_fp64phase"),
]


def _job_inputs(i, name, n, fov_deg, m, stacks, fold, precision):
    if n <= 64:
        uvw = syn.uniform_box_uvw(m, u_max=40.0, w_max=20.0, seed=100 + i)
    else:
        uvw = syn.mwa_rotation_uvw(m, 600.0) * (0.1 * n / 256)
    params = wsp.make_params(n, math.radians(fov_deg), n_stacks=stacks, fold=fold,
                             precision=precision)
    return params, uvw


@pytest.fixture(scope="module")
def jobs():
    out = []
    for i, spec in enumerate(JOBS):
        params, uvw = _job_inputs(i, *spec)
        out.append((spec, params, uvw))
    return out


def _requests(jobs, n_req, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n_req):
        j = int(rng.integers(len(jobs)))
        spec, params, uvw = jobs[j]
        fp64 = spec[6] == "fp64"
        if rng.random() < 0.5:
            data = torch.from_numpy(syn.random_image(spec[1], seed=1000 + k))
            data = data.to(torch.float64 if fp64 else torch.float32)
            reqs.append((spec[0], "forward", data))
        else:
            data = torch.from_numpy(syn.random_vis(uvw.shape[0], seed=2000 + k))
            data = data.to(torch.complex128 if fp64 else torch.complex64)
            reqs.append((spec[0], "adjoint", data))
    return reqs


def test_mixed_stream_matches_alone(jobs):
    reqs = _requests(jobs, 40, seed=7)
    # alone: one operator per job, requests one at a time on the default stream
    alone = {}
    ops = {spec[0]: wsp.Operator(params, uvw) for spec, params, uvw in jobs}
    for i, (name, kind, data) in enumerate(reqs):
        d = data.cuda()
        alone[i] = (ops[name].degrid(d) if kind == "forward" else ops[name].grid(d)).cpu()
    for op in ops.values():
        op.close()
    # mixed: all jobs resident, requests interleaved through the server
    srv = Server(hbm_budget=64 << 30)
    for spec, params, uvw in jobs:
        srv.register_job(spec[0], params, uvw)
    handles = []
    for name, kind, data in reqs:
        handles.append(srv.submit(name, kind, data.cuda()))
        srv.step()
    srv.drain()
    torch.cuda.synchronize()
    assert len(srv.done) == len(reqs)
    overlapped = 0
    for i, h in enumerate(handles):
        assert torch.equal(h.result.cpu(), alone[i]), (i, reqs[i][:2])
    # requests of different jobs were in flight together at some point
    spans = sorted((h.t_start, h.t_done) for h in handles)
    for (s0, e0), (s1, e1) in zip(spans, spans[1:]):
        overlapped += s1 < e0
    print("latency", srv.latency_percentiles(), "overlapping launches", overlapped)
    for spec, params, uvw in jobs:
        srv.retire_job(spec[0])
    assert srv.resident_bytes == 0


def test_admission_by_footprint(jobs):
    fps = [job_footprint_bytes(params, uvw) for spec, params, uvw in jobs]
    budget = max(fps) + min(fps)          # not everything fits at once
    srv = Server(hbm_budget=budget)
    for (spec, params, uvw), fp in zip(jobs, fps):
        srv.register_job(spec[0], params, uvw, footprint=fp)
    assert srv.resident_bytes <= budget
    waiting = [j.job_id for j in srv.waiting_jobs]
    assert waiting, "the budget should hold some jobs back"
    resident = [k for k, j in srv.jobs.items() if j.op is not None]
    for name in resident:
        srv.retire_job(name)
    srv.drain()
    # retiring resident jobs admits the waiting ones, within the budget
    assert srv.resident_bytes <= budget
    assert len(srv.waiting_jobs) < len(waiting)
    for name in list(srv.jobs):
        srv.retire_job(name)
    assert srv.resident_bytes == 0 and not srv.waiting_jobs


def test_oversized_job_refused(jobs):
    spec, params, uvw = jobs[0]
    srv = Server(hbm_budget=1 << 20)
    with pytest.raises(ValueError):
        srv.register_job("big", params, uvw)
