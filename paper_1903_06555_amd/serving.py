"""Served operator: continuous batching of forward / adjoint requests.

Several imaging jobs share one GPU.  A job is one
:class:`~paper_1903_06555_amd.wsp.Operator` (its kernels, stacks and plan
resident in HBM) with ``slots`` workspaces: a (grids, scratch) pair and a
stream each, so that up to ``slots`` requests of the job run at once.
Requests -- ``forward`` (y = Phi x) or ``adjoint`` (x = Re Phi^dagger y) --
arrive at any time.  The server

- admits a job when its bytes fit the budget next to the jobs already
  resident: the taps, the slots' workspaces and the library's plan
  (``wsp_footprint`` and ``wsp_plan_stats``, counted allocation by
  allocation), plus, while it is being built, the larger of its planning and
  build temporaries; a job that does not fit waits until retired jobs free
  enough;
- plans and builds an admitted job on a builder thread and a stream of its
  own, with the build that allocates nothing (``wsp_build_kernels_noalloc``),
  so the request loop never stops for it; the job takes requests once built;
- launches a request as soon as its job has a free slot (continuous
  batching: no batch boundary to wait for), so requests of one job and of
  different jobs overlap on the device;
- times each request on the device (events on its slot's stream, mapped to
  the host clock through a reference event), and reports latency (arrival to
  device completion) and throughput.

Results do not depend on the mix: every kernel on the path is deterministic
(no floating-point atomics), so a request's output is bit-identical alone
and among others, whatever slot it ran in.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import time

import numpy as np
import torch

from . import wsp


@dataclasses.dataclass
class Slot:
    workspace: tuple
    stream: torch.cuda.Stream
    request: "Request | None" = None


@dataclasses.dataclass
class Job:
    job_id: str
    params: wsp.wsp_params
    uvw: np.ndarray
    weights: np.ndarray | None = None
    op: wsp.Operator | None = None
    slots: list = dataclasses.field(default_factory=list)
    resident: int = 0            # bytes held while admitted
    transient: int = 0           # extra bytes while planning and building
    state: str = "waiting"       # waiting -> building -> ready -> retired
    build: cf.Future | None = None
    retire_when_idle: bool = False


@dataclasses.dataclass
class Request:
    req_id: int
    job_id: str
    kind: str                   # "forward" or "adjoint"
    data: torch.Tensor          # device input
    t_arrival: float
    t_start: float = 0.0        # device start, host clock
    t_done: float = 0.0         # device completion, host clock
    result: torch.Tensor | None = None
    ev_start: torch.cuda.Event | None = None
    ev_done: torch.cuda.Event | None = None
    io_bytes: int = 0

    @property
    def latency_ms(self) -> float:
        return (self.t_done - self.t_arrival) * 1e3


def job_bytes(params: wsp.wsp_params, uvw, slots: int = 2) -> tuple[int, int]:
    """(resident, transient) device bytes of a job: taps + slots x (grids +
    scratch) + the library's plan; and the larger of the planning peak above
    the plan and the build temporaries (0 with the no-alloc build, but the
    allocating bound is kept as headroom)."""
    ctx = wsp.wsp_create(params)
    try:
        dev = torch.as_tensor(np.asarray(uvw, dtype=np.float64)).cuda()
        wsp.wsp_set_uvw(ctx, dev)
        k, g, s = wsp.wsp_footprint(ctx)
        st = wsp.wsp_plan_stats(ctx)
    finally:
        wsp.wsp_destroy(ctx)
    resident = k + slots * (g + s) + st["plan_bytes"]
    transient = max(st["plan_peak_bytes"] - st["plan_bytes"], st["build_temp_bytes"])
    return resident, transient


def job_footprint_bytes(params: wsp.wsp_params, uvw, slots: int = 2) -> int:
    """Bytes a job needs at admission (resident plus transient)."""
    r, t = job_bytes(params, uvw, slots)
    return r + t


class Server:
    def __init__(self, hbm_budget: int, io_budget: int = 8 << 30, device: int = 0, slots: int = 2):
        self.hbm_budget = hbm_budget
        self.io_budget = io_budget
        self.slots = slots
        self.device = torch.device("cuda", device)
        self.jobs: dict[str, Job] = {}
        self.waiting_jobs: collections.deque[Job] = collections.deque()
        self.queue: collections.deque[Request] = collections.deque()
        self.inflight: list[Request] = []
        self.done: list[Request] = []
        self.admitted_bytes = 0      # resident + transient of admitted jobs
        self.io_inflight = 0
        self._next_id = 0
        self._builder = cf.ThreadPoolExecutor(max_workers=1)  # builds share the static workspace
        self._build_stream = torch.cuda.Stream(device=self.device)   # default priority
        # device-to-host clock reference for request timing
        self._ref = torch.cuda.Event(enable_timing=True)
        self._ref.record(torch.cuda.current_stream(self.device))
        torch.cuda.synchronize(self.device)
        self._ref_host = time.perf_counter()

    @property
    def resident_bytes(self) -> int:
        return self.admitted_bytes

    # -- jobs -------------------------------------------------------------------
    def register_job(self, job_id: str, params: wsp.wsp_params, uvw, weights=None,
                     footprint: tuple[int, int] | None = None) -> Job:
        job = Job(job_id, params, np.asarray(uvw, dtype=np.float64), weights)
        job.resident, job.transient = footprint if footprint is not None else job_bytes(params, uvw, self.slots)
        if job.resident + job.transient > self.hbm_budget:
            raise ValueError(f"job {job_id} needs {job.resident + job.transient} bytes, budget {self.hbm_budget}")
        self.jobs[job_id] = job
        self.waiting_jobs.append(job)
        self._admit_jobs()
        return job

    def retire_job(self, job_id: str):
        """Free the job's device memory once its queued and running requests are done."""
        self.jobs[job_id].retire_when_idle = True
        self._retire_idle()

    def _build(self, job: Job):
        """Builder thread: plan, bind and build with nothing allocated by the build itself."""
        torch.cuda.set_device(self.device)
        s = self._build_stream
        with torch.cuda.stream(s):
            op = wsp.Operator(job.params, job.uvw, weights=job.weights, build=False, stream=s)
            op.build_status = wsp.wsp_build_kernels_noalloc(op.ctx, s)
            slots = [Slot(op.new_workspace(), torch.cuda.Stream(device=self.device)) for _ in range(self.slots)]
        s.synchronize()
        return op, slots

    def _admit_jobs(self):
        while self.waiting_jobs:
            job = self.waiting_jobs[0]
            if self.admitted_bytes + job.resident + job.transient > self.hbm_budget:
                return
            self.waiting_jobs.popleft()
            self.admitted_bytes += job.resident + job.transient
            job.state = "building"
            job.build = self._builder.submit(self._build, job)

    def _poll_builds(self):
        for job in self.jobs.values():
            if job.state == "building" and job.build.done():
                job.op, job.slots = job.build.result()   # re-raises a build failure
                job.build = None
                job.state = "ready"
                self.admitted_bytes -= job.transient       # the temporaries are gone
                job.transient = 0

    def _retire_idle(self):
        for job in self.jobs.values():
            if (job.retire_when_idle and job.state == "ready"
                    and all(sl.request is None for sl in job.slots)
                    and not any(r.job_id == job.job_id for r in self.queue)):
                for sl in job.slots:
                    sl.stream.synchronize()
                job.op.close()
                job.op = None
                job.slots = []
                job.state = "retired"
                self.admitted_bytes -= job.resident
        self._admit_jobs()

    def wait_ready(self):
        """Block until every admitted job is built (for set-up and tests)."""
        for job in self.jobs.values():
            if job.state == "building":
                job.build.result()
        self._poll_builds()

    # -- requests ---------------------------------------------------------------
    def submit(self, job_id: str, kind: str, data: torch.Tensor) -> Request:
        if kind not in ("forward", "adjoint"):
            raise ValueError(kind)
        req = Request(self._next_id, job_id, kind, data, time.perf_counter())
        self._next_id += 1
        self.queue.append(req)
        self.step()
        return req

    def _io_bytes(self, job: Job) -> int:
        cb = 16 if job.params.precision == wsp.WSP_FP64 else 8
        return job.uvw.shape[0] * cb + job.params.n * job.params.n * cb // 2

    def _device_time(self, ev: torch.cuda.Event) -> float:
        return self._ref_host + self._ref.elapsed_time(ev) * 1e-3

    def step(self):
        """Retire finished requests and built jobs, then launch every request that can start."""
        still = []
        for r in self.inflight:
            if r.ev_done.query():
                r.t_start = self._device_time(r.ev_start)
                r.t_done = self._device_time(r.ev_done)
                job = self.jobs[r.job_id]
                for sl in job.slots:
                    if sl.request is r:
                        sl.request = None
                self.io_inflight -= r.io_bytes
                self.done.append(r)
            else:
                still.append(r)
        self.inflight = still
        self._poll_builds()
        self._retire_idle()
        pending = collections.deque()
        while self.queue:
            r = self.queue.popleft()
            job = self.jobs[r.job_id]
            io = self._io_bytes(job)
            free = [sl for sl in job.slots if sl.request is None] if job.state == "ready" else []
            if not free or self.io_inflight + io > self.io_budget:
                pending.append(r)
                continue
            self._launch(job, free[0], r, io)
        self.queue = pending

    def _launch(self, job: Job, slot: Slot, r: Request, io: int):
        slot.request = r
        r.io_bytes = io
        self.io_inflight += io
        producer = torch.cuda.current_stream(self.device)
        slot.stream.wait_stream(producer)
        with torch.cuda.stream(slot.stream):
            data = r.data
            data.record_stream(slot.stream)
            r.ev_start = torch.cuda.Event(enable_timing=True)
            r.ev_start.record(slot.stream)
            if r.kind == "forward":
                r.result = job.op.degrid(data, stream=slot.stream, workspace=slot.workspace)
            else:
                r.result = job.op.grid(data, stream=slot.stream, workspace=slot.workspace)
            r.ev_done = torch.cuda.Event(enable_timing=True)
            r.ev_done.record(slot.stream)
        self.inflight.append(r)

    def drain(self, poll_s: float = 0.0):
        while self.queue or self.inflight or any(j.state == "building" for j in self.jobs.values()):
            self.step()
            if poll_s:
                time.sleep(poll_s)

    def close(self):
        self._builder.shutdown(wait=True)

    # -- metrics ----------------------------------------------------------------
    def latency_percentiles(self):
        lat = np.array([r.latency_ms for r in self.done])
        if lat.size == 0:
            return {}
        return {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                "mean": float(lat.mean()), "n": int(lat.size)}

    def max_concurrency(self, requests=None) -> int:
        """Most requests whose device intervals [start, done] overlap at one time."""
        reqs = self.done if requests is None else requests
        ev = sorted([(r.t_start, 1) for r in reqs] + [(r.t_done, -1) for r in reqs])
        cur = best = 0
        for _, d in ev:
            cur += d
            best = max(best, cur)
        return best
