"""Served operator: continuous batching of forward / adjoint requests.

Several imaging jobs (each an :class:`~paper_1903_06555_amd.wsp.Operator`
with its kernels, stacks and FFT grids resident in HBM) share one GPU.
Requests -- ``forward`` (y = Phi x) or ``adjoint`` (x = Re Phi^dagger y) --
arrive at any time.  The server

- admits a job only if its exact HBM footprint (``wsp_footprint``) fits the
  budget next to the jobs already resident; a job that does not fit waits
  until enough resident jobs have been retired;
- keeps one stream per resident job (a job's context owns one set of grids,
  so its requests run in order on that stream), and launches a request as
  soon as its job has a free slot -- requests of different jobs overlap on
  the device, and a request that arrives while others run is admitted
  immediately (continuous batching: no batch boundary to wait for);
- bounds the bytes of request inputs/outputs in flight;
- reports per-request latency (arrival to completion) and throughput.

Results do not depend on the mix: every kernel on the path is deterministic
(no floating-point atomics), so a request's output is bit-identical alone
and among others.
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np
import torch

from . import wsp


@dataclasses.dataclass
class Job:
    job_id: str
    params: wsp.wsp_params
    uvw: np.ndarray
    weights: np.ndarray | None = None
    op: wsp.Operator | None = None
    stream: torch.cuda.Stream | None = None
    footprint: int = 0
    busy: bool = False
    retire_when_idle: bool = False


@dataclasses.dataclass
class Request:
    req_id: int
    job_id: str
    kind: str                   # "forward" or "adjoint"
    data: torch.Tensor          # device input
    t_arrival: float
    t_start: float = 0.0
    t_done: float = 0.0
    result: torch.Tensor | None = None
    done_event: torch.cuda.Event | None = None
    io_bytes: int = 0

    @property
    def latency_ms(self) -> float:
        return (self.t_done - self.t_arrival) * 1e3


def job_footprint_bytes(params: wsp.wsp_params, uvw) -> int:
    """Exact bytes a job keeps resident: taps, grids, scratch (plan excluded)."""
    ctx = wsp.wsp_create(params)
    try:
        dev = torch.as_tensor(np.asarray(uvw, dtype=np.float64)).cuda()
        wsp.wsp_set_uvw(ctx, dev)
        k, g, s = wsp.wsp_footprint(ctx)
    finally:
        wsp.wsp_destroy(ctx)
    return k + g + s


class Server:
    def __init__(self, hbm_budget: int, io_budget: int = 8 << 30, device: int = 0):
        self.hbm_budget = hbm_budget
        self.io_budget = io_budget
        self.device = torch.device("cuda", device)
        self.jobs: dict[str, Job] = {}
        self.waiting_jobs: collections.deque[Job] = collections.deque()
        self.queue: collections.deque[Request] = collections.deque()
        self.inflight: list[Request] = []
        self.done: list[Request] = []
        self.resident_bytes = 0
        self.io_inflight = 0
        self._next_id = 0

    # -- jobs -------------------------------------------------------------------
    def register_job(self, job_id: str, params: wsp.wsp_params, uvw, weights=None,
                     footprint: int | None = None) -> Job:
        job = Job(job_id, params, np.asarray(uvw, dtype=np.float64), weights)
        job.footprint = footprint if footprint is not None else job_footprint_bytes(params, uvw)
        if job.footprint > self.hbm_budget:
            raise ValueError(f"job {job_id} needs {job.footprint} bytes, budget {self.hbm_budget}")
        self.jobs[job_id] = job
        self.waiting_jobs.append(job)
        self._admit_jobs()
        return job

    def retire_job(self, job_id: str):
        """Free the job's device memory once its queued requests are served."""
        job = self.jobs[job_id]
        job.retire_when_idle = True
        self._retire_idle()

    def _admit_jobs(self):
        while self.waiting_jobs:
            job = self.waiting_jobs[0]
            if self.resident_bytes + job.footprint > self.hbm_budget:
                return
            self.waiting_jobs.popleft()
            job.stream = torch.cuda.Stream(device=self.device)   # default priority
            with torch.cuda.stream(job.stream):
                job.op = wsp.Operator(job.params, job.uvw, weights=job.weights)
            job.stream.synchronize()
            self.resident_bytes += job.footprint

    def _retire_idle(self):
        for job in self.jobs.values():
            if (job.retire_when_idle and job.op is not None and not job.busy
                    and not any(r.job_id == job.job_id for r in self.queue)):
                job.stream.synchronize()
                job.op.close()
                job.op = None
                self.resident_bytes -= job.footprint
        self._admit_jobs()

    # -- requests ---------------------------------------------------------------
    def submit(self, job_id: str, kind: str, data: torch.Tensor) -> Request:
        if kind not in ("forward", "adjoint"):
            raise ValueError(kind)
        req = Request(self._next_id, job_id, kind, data, time.perf_counter())
        self._next_id += 1
        self.queue.append(req)
        self.step()
        return req

    def _io_bytes(self, job: Job, kind: str) -> int:
        cb = 16 if job.params.precision == wsp.WSP_FP64 else 8
        n = job.params.n
        m = job.uvw.shape[0]
        return m * cb + n * n * cb // 2

    def step(self):
        """Retire finished requests, then launch every request that can start."""
        still = []
        now = time.perf_counter()
        for r in self.inflight:
            if r.done_event.query():
                r.t_done = now
                self.jobs[r.job_id].busy = False
                self.io_inflight -= r.io_bytes
                self.done.append(r)
            else:
                still.append(r)
        self.inflight = still
        self._retire_idle()
        pending = collections.deque()
        while self.queue:
            r = self.queue.popleft()
            job = self.jobs[r.job_id]
            io = self._io_bytes(job, r.kind)
            if job.op is None or job.busy or self.io_inflight + io > self.io_budget:
                pending.append(r)
                continue
            self._launch(job, r, io)
        self.queue = pending

    def _launch(self, job: Job, r: Request, io: int):
        job.busy = True
        r.io_bytes = io
        self.io_inflight += io
        r.t_start = time.perf_counter()
        producer = torch.cuda.current_stream(self.device)
        job.stream.wait_stream(producer)
        with torch.cuda.stream(job.stream):
            data = r.data
            data.record_stream(job.stream)
            if r.kind == "forward":
                r.result = job.op.degrid(data)
            else:
                r.result = job.op.grid(data)
            r.done_event = torch.cuda.Event()
            r.done_event.record(job.stream)
        self.inflight.append(r)

    def drain(self, poll_s: float = 0.0):
        while self.queue or self.inflight:
            self.step()
            if poll_s:
                time.sleep(poll_s)

    # -- metrics ----------------------------------------------------------------
    def latency_percentiles(self):
        lat = np.array([r.latency_ms for r in self.done])
        if lat.size == 0:
            return {}
        return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                "mean": float(lat.mean()), "n": int(lat.size)}
