"""Served operator: continuous batching on the device.

Jobs of the served workload's sizes (512^2 to 4096^2 images, 1 to 4
w-stacks, FP32 and FP64) share the GPU.  Checks: every request's result is
bit-identical alone (its job's operator on its own) and in a mixed stream
through the server; requests of different jobs, and two requests of one
job (its two slots), run at the same time on the device (their device
intervals, from events on the slots' streams, overlap); admission follows
the reported bytes; and a job being planned and built on the builder thread
does not stop requests of the other jobs from completing.
"""
import math
import time

import numpy as np
import pytest
import torch

from paper_1903_06555_amd import synthetic as syn
from paper_1903_06555_amd import wsp
from paper_1903_06555_amd.serving import Server, job_bytes, job_footprint_bytes

pytestmark = pytest.mark.gpu

JOBS = [  # (name, n, fov_deg, m, stacks, fold, precision)
    ("a", 512, 25.0, 100_000, 2, True, "fp32_fp64phase"),
    ("b", 1024, 25.0, 200_000, 4, True, "fp32_fp64phase"),
    ("c", 2048, 25.0, 150_000, 1, False, "fp64"),
    ("d", 4096, 25.0, 100_000, 2, True, "fp32_fp64phase"),
]


def _job_inputs(spec):
    name, n, fov_deg, m, stacks, fold, precision = spec
    uvw = syn.mwa_rotation_uvw(m, 1800.0)
    params = wsp.make_params(n, math.radians(fov_deg), n_stacks=stacks, fold=fold, precision=precision)
    return params, uvw


@pytest.fixture(scope="module")
def jobs():
    return [(spec, *_job_inputs(spec)) for spec in JOBS]


def _requests(jobs, n_req, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n_req):
        spec, params, uvw = jobs[int(rng.integers(len(jobs)))]
        fp64 = spec[6] == "fp64"
        if rng.random() < 0.5:
            data = torch.from_numpy(syn.random_image(spec[1], seed=1000 + k))
            reqs.append((spec[0], "forward", data.to(torch.float64 if fp64 else torch.float32)))
        else:
            data = torch.from_numpy(syn.random_vis(uvw.shape[0], seed=2000 + k))
            reqs.append((spec[0], "adjoint", data.to(torch.complex128 if fp64 else torch.complex64)))
    return reqs


def _overlap(a, b):
    return a.t_start < b.t_done and b.t_start < a.t_done


def test_mixed_stream_matches_alone_and_overlaps(jobs):
    reqs = _requests(jobs, 32, seed=7)
    alone = {}
    for spec, params, uvw in jobs:
        op = wsp.Operator(params, uvw)
        for i, (name, kind, data) in enumerate(reqs):
            if name == spec[0]:
                d = data.cuda()
                alone[i] = (op.degrid(d) if kind == "forward" else op.grid(d)).cpu()
        op.close()
        torch.cuda.empty_cache()
    srv = Server(hbm_budget=200 << 30, slots=2)
    for spec, params, uvw in jobs:
        srv.register_job(spec[0], params, uvw)
    srv.wait_ready()
    inputs = [data.cuda() for _, _, data in reqs]
    torch.cuda.synchronize()
    handles = [srv.submit(name, kind, d) for (name, kind, _), d in zip(reqs, inputs)]
    srv.drain()
    torch.cuda.synchronize()
    assert len(srv.done) == len(reqs)
    for i, h in enumerate(handles):
        assert torch.equal(h.result.cpu(), alone[i]), (i, reqs[i][:2])
    conc = srv.max_concurrency(handles)
    cross = sum(_overlap(a, b) for i, a in enumerate(handles) for b in handles[i + 1:] if a.job_id != b.job_id)
    same = sum(_overlap(a, b) for i, a in enumerate(handles) for b in handles[i + 1:] if a.job_id == b.job_id)
    print(f"latency {srv.latency_percentiles()}; max concurrency {conc}; overlapping pairs across jobs "
          f"{cross}, within a job {same}", flush=True)
    assert conc >= 3 and cross > 0 and same > 0
    for spec, params, uvw in jobs:
        srv.retire_job(spec[0])
    assert srv.resident_bytes == 0
    srv.close()


def test_admission_by_reported_bytes(jobs):
    sizes = [job_bytes(params, uvw, 2) for spec, params, uvw in jobs]
    totals = [r + t for r, t in sizes]
    budget = max(totals) + min(totals)          # not everything fits at once
    srv = Server(hbm_budget=budget, slots=2)
    for (spec, params, uvw), sz in zip(jobs, sizes):
        srv.register_job(spec[0], params, uvw, footprint=sz)
    assert srv.resident_bytes <= budget
    waiting = [j.job_id for j in srv.waiting_jobs]
    assert waiting, "the budget should hold some jobs back"
    srv.wait_ready()
    # an admitted job's device memory is what was reserved for it: its operator's
    # buffers, the slots' workspaces and the plan the library reports
    for job in srv.jobs.values():
        if job.state == "ready":
            fp = job.op.footprint
            held = (fp["kernel_bytes"] + 2 * (fp["grid_bytes"] + fp["scratch_bytes"]) +
                    job.op.plan_stats()["plan_bytes"])
            assert held == job.resident, (job.job_id, held, job.resident)
    for name in [k for k, j in srv.jobs.items() if j.state == "ready"]:
        srv.retire_job(name)
    srv.drain()
    assert srv.resident_bytes <= budget
    assert len(srv.waiting_jobs) < len(waiting)
    for name in list(srv.jobs):
        srv.retire_job(name)
    srv.drain()
    for name in list(srv.jobs):
        srv.retire_job(name)
    assert srv.resident_bytes == 0 and not srv.waiting_jobs
    srv.close()


def test_requests_complete_while_a_job_builds(jobs):
    spec, params, uvw = jobs[0]
    srv = Server(hbm_budget=200 << 30, slots=2)
    srv.register_job("small", params, uvw)
    srv.wait_ready()
    x = torch.from_numpy(syn.random_image(spec[1], seed=5)).float().cuda()
    # a large job: planning and building take a good fraction of a second
    big_params = wsp.make_params(2048, math.radians(25.0), n_stacks=8, fold=True)
    srv.register_job("big", big_params, syn.mwa_rotation_uvw(3_000_000, 1800.0))
    assert srv.jobs["big"].state == "building"
    done_while_building = 0
    t0 = time.perf_counter()
    while srv.jobs["big"].state == "building" and time.perf_counter() - t0 < 120:
        n_before = len(srv.done)
        srv.submit("small", "forward", x)
        srv.step()
        if srv.jobs["big"].state == "building":
            done_while_building += len(srv.done) - n_before
    srv.drain()
    print(f"{done_while_building} small requests completed while the big job was being built", flush=True)
    assert srv.jobs["big"].state == "ready" and srv.jobs["big"].op.build_status == wsp.WSP_OK
    assert done_while_building >= 5
    for name in list(srv.jobs):
        srv.retire_job(name)
    srv.drain()
    srv.close()


def test_oversized_job_refused(jobs):
    spec, params, uvw = jobs[0]
    srv = Server(hbm_budget=1 << 20)
    with pytest.raises(ValueError):
        srv.register_job("big", params, uvw)
    assert job_footprint_bytes(params, uvw) > (1 << 20)
    srv.close()
