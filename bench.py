"""Benchmark: degrid + grid throughput with per-visibility exact w-kernels.

One step is one application of the measurement operator and its adjoint
(y = Phi x, then x' = Re Phi^dagger y) over all visibilities, with the
kernels already built and resident in HBM (the metric's definition).
Folding, k-means, sorting and the kernel build run once before the timed
region and are reported separately.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

The default line is the one-GPU share of the hybrid method: 4096^2 image,
25 degree field, 2.5e7 MWA-like visibilities folded and split into 16
w-stacks.  It carries, as extra fields, the same workload on the all-FP64
path and the 1024^2 single-stack workload (mean support 87).  Prints one
JSON line.  Inputs are seeded synthetic MWA-like data (the paper's Fornax A
visibilities are not available).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s


def log(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mwa_4096_16_stacks")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra fields (all-FP64 path, 1024^2 single-stack workload)")
    ap.add_argument("--cpu-workers", type=int, default=0, help="CPU-baseline processes (0: all host cores, <= 16)")
    ap.add_argument("--precision", default=None, help="override: fp32_fp64phase or fp64")
    ap.add_argument("--m-vis", type=int, default=None, help="override visibility count (debug)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1600)
    ap.add_argument("--stacks", type=int, default=None, help="override the workload's w-stack count")
    ap.add_argument("--fold", type=int, choices=[0, 1], default=None,
                    help="override the workload's conjugate-symmetry folding")
    ap.add_argument("--kernels", default="exact", choices=["exact", "planes"],
                    help="exact per-visibility taps, or taps interpolated from 1-D w-planes")
    ap.add_argument("--band-rows", type=int, default=0, choices=[0, 8, 16],
                    help="exact mode: tile rows per band of the tap layout (0: the library's choice)")
    ap.add_argument("--item-taps", type=int, default=0,
                    help="exact mode: taps per tile work item (0: the library's default, 2^19)")
    ap.add_argument("--tap-layout", default="auto", choices=["auto", "runs", "interleaved"],
                    help="exact mode: tap layout (auto: interleaved when runs are short)")
    ap.add_argument("--mode", default="operator", choices=["operator", "copy", "serving", "build"],
                    help="operator: the metric; copy: a plain 2 GiB device copy used to "
                         "calibrate rocprofv3 FETCH_SIZE / WRITE_SIZE readings; serving: "
                         "Poisson request stream from several imaging jobs")
    ap.add_argument("--serve-jobs", type=int, default=8)
    ap.add_argument("--serve-mmin", type=float, default=1e5)
    ap.add_argument("--serve-mmax", type=float, default=2e7)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-load", type=float, default=0.75)
    ap.add_argument("--serve-budget-gb", type=float, default=240.0)
    return ap.parse_args()


def traffic_file(workload: str, precision: str) -> str:
    suffix = "" if precision == "fp32_fp64phase" else f"_{precision}"
    return os.path.join(ROOT, "profiles", f"traffic_{workload}{suffix}.json")
TRAFFIC_SOURCES = ("paper_1903_06555_amd/csrc/apply.hip", "paper_1903_06555_amd/csrc/wsp_internal.h",
                   "paper_1903_06555_amd/csrc/plan.hip")


def source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str, m: int, precision: str):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    readings (calibrated on a plain copy), or None if they were taken on other
    kernel sources, another workload or another precision."""
    try:
        with open(traffic_file(workload, precision)) as fh:
            rec = json.load(fh)
    except OSError:
        return None
    if rec.get("source_sha256") != source_digest() or rec.get("workload") != workload \
            or rec.get("m_vis") != m or rec.get("precision", "fp32_fp64phase") != precision:
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["fetch_bytes"] + k["write_bytes"]


def algorithmic_bytes(stage: str, taps: int, m: int, touched_cells: int, cb: int) -> int:
    """Bytes one launch of a stage must move at minimum.

    degrid: every tap once, every distinct touched grid cell once (cb
    bytes), per visibility its base (8 B), weight (4 B) and output (cb B).
    grid: the same taps and per-visibility bytes with the visibility read
    instead of written, and a read-modify-write of every touched cell (2 cb
    bytes).  Cells no tap touches are not counted.
    """
    per_vis = 8 + 4 + cb
    cell_bytes = cb if stage == "degrid" else 2 * cb
    return taps * cb + m * per_vis + touched_cells * cell_bytes


# w-plane mode: FP32 operations per tap of the interpolation and the
# multiply-add, counting an FMA as two (distance 6, lattice index 3, bilinear
# complex interpolation 18, conjugation 1, complex multiply-add 8)
PLANE_FLOPS_PER_TAP = 36
# VALU FP32 peak without packed FP32 instructions (not used by this build):
# 256 CUs x 64 lanes x 2 (FMA) x 2.4 GHz
VALU_FP32_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _oracle_chunk(task):
    """One CPU-baseline process: the oracle's degrid + grid for one w-stack.

    Times the stack's fixed part (taper, zero pad and FFT; inverse FFT, crop
    and untaper: oracle stack_grid and finish_adjoint) and, apart from it,
    the per-visibility part on a chunk of the stack's visibilities (oracle
    degrid_stack and grid_stack), with random taps of the visibilities' true
    shapes in the oracle's kernel cache (kernel construction is not part of
    a step)."""
    name, uvw, labels, centres, seed = task
    import math as _m

    from oracle import operator, wkernel
    from paper_1903_06555_amd import synthetic as syn
    wl = syn.WORKLOADS[name]
    geom = wkernel.Geometry(n=wl.n, fov=_m.radians(wl.fov_deg))
    ref = operator.StackedOperator(geom, uvw, n_stacks=centres.size, fold=wl.fold, labels=labels,
                                   centres=centres)
    rng = np.random.default_rng(seed)
    for p in range(ref.m):
        jp = int(ref.jp[p])
        u0, v0, _ = wkernel.tap_geometry(ref.u_pix[p], ref.v_pix[p], jp)
        ref._kernels[p] = (u0, v0, rng.normal(size=(jp, jp)) + 1j * rng.normal(size=(jp, jp)))
    k = int(labels[0])
    x = syn.workload_sky(wl)
    y = syn.random_vis(ref.m, seed)
    members = np.arange(ref.m)
    t0 = time.perf_counter()
    grid = ref.stack_grid(x, k)
    ref.finish_adjoint(np.zeros_like(grid), k)
    t1 = time.perf_counter()
    out = np.zeros(ref.m, dtype=np.complex128)
    ref.degrid_stack(grid, members, out)
    ref.grid_stack(y, members)
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1, ref.m


def cpu_baseline(wl, uvw, sample_n: int, workers: int):
    """The FP64 oracle's degrid + grid on the host's cores, on a bounded sample.

    The oracle's stack assignment (3 Lloyd iterations of Algorithm 1: enough
    for the supports' distribution) sorts the visibilities into stacks.
    ``workers`` processes (spawned, so no GPU context is inherited) run at
    once, each on one stack: the stack's fixed part (taper, zero pad, FFT and
    their adjoints) and, timed apart, the degrid + grid of a chunk of its
    visibilities at uniform quantiles of J_p.  Kernel construction is
    outside a step, so the oracle's kernel cache holds random taps of each
    visibility's true shape.  A step on ``workers`` cores is then
    extrapolated as ceil(K / workers) fixed parts plus M visibilities' costs
    shared over the cores (both as measured while all processes ran
    together).
    """
    import concurrent.futures as cf
    import multiprocessing as mp

    from oracle import stacking, wkernel
    geom = wkernel.Geometry(n=wl.n, fov=math.radians(wl.fov_deg))
    folded, _ = stacking.fold(uvw) if wl.fold else (uvw, None)
    labels, centres, _ = stacking.kmeans_w(folded[:, 2], wl.n_stacks, 1e-3, 3)
    K = centres.size
    jp = wkernel.support(folded[:, 2] - centres[labels], geom)
    stacks = [int(k) for k in np.linspace(0, K - 1, workers).round().astype(int)]
    per = max(2, sample_n // workers)
    tasks = []
    for i, k in enumerate(stacks):
        members = np.flatnonzero(labels == k)
        order = members[np.argsort(jp[members], kind="stable")]
        rot = i * 7919 % max(1, order.size)  # workers on the same stack take different visibilities
        pick = np.unique((np.linspace(0, order.size - 1, min(per, order.size)).astype(np.int64) + rot) % order.size)
        idx = order[pick]
        tasks.append((wl.name, uvw[idx], labels[idx], centres, 100 + i))
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_oracle_chunk, tasks))
    wall = time.perf_counter() - t0
    fixed = float(np.mean([r[0] for r in res]))
    per_vis = float(np.sum([r[1] for r in res]) / np.sum([r[2] for r in res]))
    m = uvw.shape[0]
    t_step = math.ceil(K / workers) * fixed + m * per_vis / workers
    n_s = sum(r[2] for r in res)
    return {
        "value": m / t_step / 1e6,
        "unit": "Mvis/s",
        "cores": workers,
        "kind": "oracle",
        "host_cpu_count": os.cpu_count(),
        "host_cpu_model": host_cpu_model(),
        "sample": (f"{n_s} visibilities in {len(set(stacks))} of {K} stacks, {workers} processes at once, "
                   f"each one stack's fixed part (FFT, taper, crop) and, timed apart, degrid + grid of "
                   f"its visibilities at uniform J_p quantiles; oracle with random taps of the "
                   f"true shapes (kernel construction excluded); a step on {workers} cores extrapolated as "
                   f"ceil(K/{workers}) fixed parts plus all {m} visibilities' cost over {workers} cores"),
        "per_vis_us_concurrent": per_vis * 1e6,
        "fixed_s_per_stack_concurrent": fixed,
        "extrapolated_step_s": t_step,
        "measure_wall_s": wall,
    }


def copy_calibration(steps: int):
    """A plain device-to-device copy of known size (counter calibration)."""
    import torch
    nbytes = 2 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    print(json.dumps({"mode": "copy", "bytes_read_per_launch": nbytes,
                      "bytes_written_per_launch": nbytes, "launches": steps,
                      "GB_s": 2 * nbytes / dt / 1e9}))


def serving(args):
    """Continuous-batching server fed by a seeded Poisson stream (see serving.py).

    8 jobs (512^2 - 4096^2 images, 1e5 - 2e7 visibilities log-uniform, 1 - 16
    stacks, folded when K > 1), two slots each.  The offered load is 75% of the
    unbatched capacity (each request alone, back to back); latency is arrival
    to device completion.  Also: the same requests queued at once (saturated),
    the unbatched rate, and the plain unbatched all-FP64 path's rate."""
    import torch

    from paper_1903_06555_amd import synthetic as syn
    from paper_1903_06555_amd import wsp
    from paper_1903_06555_amd.serving import Server

    rng = np.random.default_rng(5)
    specs = []
    for j in range(args.serve_jobs):
        n = int(rng.choice([512, 1024, 2048, 4096]))
        m = int(np.exp(rng.uniform(np.log(args.serve_mmin), np.log(args.serve_mmax))))
        k = int(rng.integers(1, 17))
        specs.append((f"job{j}", n, m, k, k > 1))
    # one MWA-like track per job (30 min of rotation), first m visibilities
    base = syn.mwa_rotation_uvw(int(max(s[2] for s in specs)), 1800.0)
    srv = Server(hbm_budget=int(args.serve_budget_gb * 2**30), slots=2)
    t0 = time.perf_counter()
    refused = []
    for name, n, m, k, fold in specs:
        params = wsp.make_params(n, math.radians(25.0), n_stacks=k, fold=fold)
        try:
            srv.register_job(name, params, base[:m])
        except ValueError:
            refused.append(name)
        log(f"registered {name}: N={n} M={m} K={k} ({time.perf_counter() - t0:.1f} s)")
    srv.wait_ready()
    log(f"all admitted jobs built ({time.perf_counter() - t0:.1f} s)")
    if srv.waiting_jobs:
        raise RuntimeError("jobs left waiting at start; raise --serve-budget-gb")
    live = [sp for sp in specs if sp[0] not in refused]
    dev = torch.device("cuda", 0)
    inputs = {}
    for name, n, m, k, fold in live:
        inputs[name] = (torch.from_numpy(syn.point_source_sky(n, 200, "exp", 7)).float().to(dev),
                        torch.from_numpy(syn.random_vis(m, 8)).to(torch.complex64).to(dev))
    # capacity of the unbatched path: each request alone, back to back
    t_alone = {}
    for name, n, m, k, fold in live:
        op = srv.jobs[name].op
        for kind in ("forward", "adjoint"):
            x, y = inputs[name]
            torch.cuda.synchronize()
            tt = time.perf_counter()
            for _ in range(3):
                op.degrid(x) if kind == "forward" else op.grid(y)
            torch.cuda.synchronize()
            t_alone[(name, kind)] = (time.perf_counter() - tt) / 3
    mean_service = float(np.mean(list(t_alone.values())))
    rate = args.serve_load / mean_service
    arrivals = np.cumsum(rng.exponential(1.0 / rate, args.serve_requests))
    plan = [(live[int(rng.integers(len(live)))][0], ("forward", "adjoint")[i % 2])
            for i in range(args.serve_requests)]
    log(f"offered load {args.serve_load:.2f} of unbatched capacity: {rate:.1f} req/s")
    torch.cuda.synchronize()
    start = time.perf_counter()
    i = 0
    reqs = []
    while i < len(plan) or srv.queue or srv.inflight:
        now = time.perf_counter() - start
        while i < len(plan) and arrivals[i] <= now:
            name, kind = plan[i]
            x, y = inputs[name]
            reqs.append(srv.submit(name, kind, x if kind == "forward" else y))
            i += 1
        srv.step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - start
    vis = sum(srv.jobs[r.job_id].uvw.shape[0] for r in reqs)
    unbatched_s = sum(t_alone[(r.job_id, r.kind)] for r in reqs)
    lat = srv.latency_percentiles()
    conc = srv.max_concurrency(reqs)
    for r in reqs:
        r.result = None
    # saturated: the same requests all queued at once (closed loop)
    srv.done = []
    torch.cuda.synchronize()
    start = time.perf_counter()
    sat = []
    for name, kind in plan:
        x, y = inputs[name]
        sat.append(srv.submit(name, kind, x if kind == "forward" else y))
    srv.drain()
    torch.cuda.synchronize()
    wall_sat = time.perf_counter() - start
    conc_sat = srv.max_concurrency(sat)
    for r in sat:
        r.result = None
    log(f"saturated: {len(sat)} requests in {wall_sat:.2f} s")
    for name in list(srv.jobs):
        if srv.jobs[name].state == "ready":
            srv.retire_job(name)
    srv.close()
    # the plain unbatched FP64 path on the same request plan, one job at a time
    t64 = {}
    for name, n, m, k, fold in live:
        params = wsp.make_params(n, math.radians(25.0), n_stacks=k, fold=fold, precision="fp64")
        op = wsp.Operator(params, base[:m])
        x, y = inputs[name]
        x, y = x.double(), y.to(torch.complex128)
        for kind in ("forward", "adjoint"):
            torch.cuda.synchronize()
            tt = time.perf_counter()
            for _ in range(3):
                op.degrid(x) if kind == "forward" else op.grid(y)
            torch.cuda.synchronize()
            t64[(name, kind)] = (time.perf_counter() - tt) / 3
        op.close()
        torch.cuda.empty_cache()
        log(f"fp64 baseline {name} done")
    unbatched64_s = sum(t64[(r.job_id, r.kind)] for r in reqs)
    print(json.dumps({
        "metric": "served operator requests: p50/p99 latency and Mvis/s",
        "mode": "serving", "requests": len(reqs), "wall_s": wall,
        "value": vis / wall / 1e6, "unit": "Mvis/s",
        "latency_ms": lat, "latency_clock": "arrival (host) to device completion (event on the slot's stream)",
        "offered_load": args.serve_load, "slots_per_job": 2,
        "max_concurrent_requests": conc, "max_concurrent_requests_saturated": conc_sat,
        "saturated_mvis_per_s": vis / wall_sat / 1e6,
        "unbatched_mvis_per_s": vis / unbatched_s / 1e6,
        "unbatched_fp64_mvis_per_s": vis / unbatched64_s / 1e6,
        "jobs": [{"name": a, "n": b, "m": c, "stacks": d} for a, b, c, d, _ in live],
        "refused": refused, "dtype": "f32", "data": "synthetic",
    }))


def build_rate(args):
    """Kernel construction throughput (set-up and build, no operator steps)."""
    import torch

    from paper_1903_06555_amd import synthetic as syn
    from paper_1903_06555_amd import wsp

    wl = syn.WORKLOADS[args.workload]
    m = args.m_vis or wl.m_vis
    precision = args.precision or wl.precision
    n_stacks = args.stacks or wl.n_stacks
    fold = wl.fold if args.fold is None else bool(args.fold)
    uvw = syn.workload_uvw(wl, m)
    params = wsp.make_params(wl.n, math.radians(wl.fov_deg), n_stacks=n_stacks, fold=fold,
                             precision=precision)
    # a configuration whose exact taps exceed the device memory is reported by
    # its footprint (e.g. one w-stack without folding on a wide field)
    ctx = wsp.wsp_create(params)
    try:
        wsp.wsp_set_uvw(ctx, torch.as_tensor(uvw).cuda())
        kb, gb, sb = wsp.wsp_footprint(ctx)
        jp_all = np.empty(m, dtype=np.int32)
        wsp.wsp_get_support(ctx, jp_all)
    finally:
        wsp.wsp_destroy(ctx)
    free = torch.cuda.mem_get_info()[0]
    if kb + gb + sb > 0.95 * free:
        print(json.dumps({
            "metric": "w-projection kernels built per second (adaptive quadrature, tol 1e-6)",
            "mode": "build", "value": None, "unit": "vis/s", "fits": False,
            "config": {"workload": wl.name, "n": wl.n, "m_vis": m, "n_stacks": n_stacks,
                       "fold": fold, "precision": precision},
            "kernel_bytes": kb, "grid_bytes": gb, "scratch_bytes": sb, "device_free_bytes": free,
            "taps": int(np.sum(jp_all.astype(np.int64) ** 2)), "mean_jp": float(jp_all.mean()),
            "max_jp": int(jp_all.max()),
        }))
        return
    t0 = time.perf_counter()
    op = wsp.Operator(params, uvw, build=False)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    _, _, iters = op.stacks()
    log(f"plan (fold, k-means {iters} iterations, sort, tile lists) {t_plan:.2f} s")
    t0 = time.perf_counter()
    op.build(part=max(1, m // 10),
             progress=lambda d, n: log(f"built {d}/{n} kernels, {time.perf_counter() - t0:.1f} s"))
    t_build = time.perf_counter() - t0
    jp, _ = op.support()
    panels, capped = op.quad_stats()
    print(json.dumps({
        "metric": "w-projection kernels built per second (adaptive quadrature, tol 1e-6)",
        "mode": "build", "value": m / t_build, "unit": "vis/s", "dtype": "f32" if precision != "fp64" else "f64",
        "config": {"workload": wl.name, "n": wl.n, "m_vis": m, "n_stacks": n_stacks,
                   "fold": fold, "precision": precision},
        "build_s": t_build, "plan_s": t_plan, "kmeans_iterations": iters,
        "taps": int(np.sum(jp.astype(np.int64) ** 2)), "mean_jp": float(jp.mean()),
        "max_jp": int(jp.max()), "quad_panels": panels, "quad_capped": capped,
        "paper_context": "126.6e6 visibilities in 15 min on 50 nodes x 16 Xeon cores "
                         "(140.7e3 vis/s), Sec. 4",
    }))
    op.close()


def run_operator(wl, precision: str, kernels: str, steps: int, warmup: int, m_override=None,
                 want_y: bool = False, band_rows: int = 0, tap_layout: str = "auto", item_taps: int = 0):
    """Plan, build and time `steps` operator steps of one workload; returns a dict."""
    import torch

    from paper_1903_06555_amd import synthetic as syn
    from paper_1903_06555_amd import wsp

    m = m_override or wl.m_vis
    uvw = syn.workload_uvw(wl, m)
    x_np = syn.workload_sky(wl)
    dev = torch.device("cuda", 0)
    fp64 = precision == "fp64"
    rdt = torch.float64 if fp64 else torch.float32
    cdt = torch.complex128 if fp64 else torch.complex64
    cb = 16 if fp64 else 8
    planes = kernels == "planes"
    params = wsp.make_params(wl.n, math.radians(wl.fov_deg), n_stacks=wl.n_stacks, fold=wl.fold,
                             precision=precision, kernels=kernels, band_rows=band_rows,
                             tap_layout=tap_layout, item_taps=item_taps)
    t0 = time.perf_counter()
    op = wsp.Operator(params, uvw, build=False)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    log(f"{wl.name} {precision}: plan done in {t_plan:.1f} s ({m} visibilities)")
    t0 = time.perf_counter()
    op.build(part=max(1, m // 5),
             progress=lambda d, n: log(f"built {d}/{n} kernels, {time.perf_counter() - t0:.1f} s"))
    t_build = time.perf_counter() - t0
    panels, capped = op.quad_stats()
    st = op.plan_stats()
    taps = int(st["taps"])

    x = torch.from_numpy(x_np).to(dev, rdt)
    y = torch.empty(m, dtype=cdt, device=dev)
    xo = torch.empty((wl.n, wl.n), dtype=rdt, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        op.degrid(x, out=y)
        op.grid(y, out=xo)
    torch.cuda.synchronize()
    wsp.wsp_set_timing(op.ctx, True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        starts[k].record(stream)
        op.degrid(x, out=y)
        op.grid(y, out=xo)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = wsp.wsp_stage_times(op.ctx)
    wsp.wsp_set_timing(op.ctx, False)
    lat = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])
    ms_per_step = wall * 1e3 / steps
    log(f"{wl.name} {precision}: timed {steps} steps, {ms_per_step:.2f} ms/step")

    per_launch = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    dom = "degrid" if per_launch["degrid"] >= per_launch["grid"] else "grid"
    lanes = int(st["tap_layout"]) == 2
    grid_runs = 2 * int(st["long_taps"]) > taps
    stage_kernels = {"degrid": ("k_degrid_lanes" if lanes else "k_degrid_class") + " + k_degrid_reduce_runs",
                     "grid": "k_prep_vis + " + ("k_grid_lanes" if lanes else
                                                "k_grid_runs" if grid_runs else "k_prep_runs + k_grid_class")
                             + " + k_reduce_tiles"}
    if planes:
        flops = PLANE_FLOPS_PER_TAP * taps
        achieved_t = flops / (per_launch[dom] * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": dom, "achieved": achieved_t, "peak": VALU_FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved_t / VALU_FP32_PEAK_TFLOPS,
                    "traffic": measured_traffic(dom, wl.name + "_planes", m, precision),
                    "algorithmic_flops": flops, "flops_per_tap": PLANE_FLOPS_PER_TAP,
                    "lattice_bytes": op.footprint["kernel_bytes"], "avg_launch_ms": per_launch[dom]}
    else:
        fracs = {}
        for stg in ("degrid", "grid"):
            alg = algorithmic_bytes(stg, taps, m, int(st["touched_cells"]), cb)
            fracs[stg] = (alg, alg / (per_launch[stg] * 1e-3) / 1e9)
        alg, achieved = fracs[dom]
        roofline = {"bound": "hbm", "kernel": dom, "kernels": stage_kernels[dom], "achieved": achieved,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "traffic": measured_traffic(dom, wl.name, m, precision),
                    "algorithmic_bytes": alg, "avg_launch_ms": per_launch[dom],
                    "other": {k: {"frac": v[1] / HBM_PEAK_GBS, "algorithmic_bytes": v[0],
                                  "avg_launch_ms": per_launch[k]} for k, v in fracs.items() if k != dom}}
    out = {
        "value": m / (ms_per_step * 1e-3) / 1e6,
        "ms_per_step": ms_per_step,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "steps": steps},
        "roofline": roofline,
        "stages_ms_per_launch": per_launch,
        "config": {"workload": wl.name, "n": wl.n, "fov_deg": wl.fov_deg, "m_vis": m,
                   "n_stacks": wl.n_stacks, "fold": wl.fold, "precision": precision,
                   "oversample": params.oversample, "kb_support": params.kb_support,
                   **({"kernels": "planes", "plane_dq": 1 / 64, "plane_dw": 1 / 16} if planes else {})},
        "setup": {"plan_s": t_plan, "build_s": t_build, "build_mvis_per_s": m / t_build / 1e6,
                  "kernel_bytes": op.footprint["kernel_bytes"], "taps": taps,
                  "rms_jp": math.sqrt(taps / m), "max_jp": int(st["max_support"]),
                  "entries": int(st["entries"]), "runs": int(st["runs"]), "band_rows": int(st["band_rows"]),
                  "tap_layout": {1: "runs", 2: "interleaved"}.get(int(st["tap_layout"]), "planes"),
                  "lanes_busy": (taps / (64 * int(st["group_steps"])) if int(st["group_steps"]) else None),
                  "classes": int(st["classes"]), "long_taps": int(st["long_taps"]),
                  "fft": "lds" if int(st["fft_lds"]) else "library", "fft_rows": int(st["fft_rows"]),
                  "items": int(st["items"]),
                  "tiles": int(st["tiles"]), "split_tiles": int(st["split_tiles"]),
                  "touched_cells": int(st["touched_cells"]), "plan_bytes": int(st["plan_bytes"]),
                  "kmeans_iterations": int(st["kmeans_iterations"]),
                  "quad_panels": panels, "quad_capped": capped},
        "dtype": "f64" if fp64 else "f32",
    }
    if want_y:
        out["_uvw"] = uvw
    op.close()
    del x, y, xo, op
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.mode == "copy":
        copy_calibration(args.steps)
        return
    if args.mode == "serving":
        serving(args)
        return
    if args.mode == "build":
        build_rate(args)
        return

    from paper_1903_06555_amd import synthetic as syn

    wl = syn.WORKLOADS[args.workload]
    precision = args.precision or wl.precision
    head = run_operator(wl, precision, args.kernels, args.steps, args.warmup, args.m_vis, want_y=True,
                        band_rows=args.band_rows, tap_layout=args.tap_layout, item_taps=args.item_taps)
    uvw = head.pop("_uvw")
    planes = args.kernels == "planes"
    result = {
        "metric": ("Mvis/s degrid+grid with w-kernels interpolated on the fly from 1-D w-planes; "
                   "p50/p99 operator latency" if planes else
                   "Mvis/s degrid+grid with per-vis exact w-kernels; p50/p99 operator latency"),
        "value": head["value"],
        "unit": "Mvis/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic",
        "config": head["config"],
        "latency_ms": head["latency_ms"],
        "roofline": head["roofline"],
        "stages_ms_per_launch": head["stages_ms_per_launch"],
        "setup": head["setup"],
    }
    if not args.no_extras and not planes and args.m_vis is None:
        # the same workload on the plain all-FP64 path, and the single-stack workload
        alt = "fp64" if precision != "fp64" else "fp32_fp64phase"
        r = run_operator(wl, alt, "exact", min(args.steps, 50), args.warmup)
        result["all_fp64_path" if alt == "fp64" else "fp32_path"] = {
            "value": r["value"], "unit": "Mvis/s", "ms_per_step": r["ms_per_step"],
            "latency_ms": r["latency_ms"], "dtype": r["dtype"], "workload": wl.name,
            "roofline_frac": r["roofline"]["frac"], "roofline_kernel": r["roofline"]["kernel"],
            "throughput_ratio_fp32_over_fp64": (head["value"] / r["value"] if alt == "fp64"
                                                else r["value"] / head["value"])}
        other = "mwa_1024_single_stack" if wl.name != "mwa_1024_single_stack" else "mwa_4096_16_stacks"
        r = run_operator(syn.WORKLOADS[other], syn.WORKLOADS[other].precision, "exact", args.steps, args.warmup)
        result[other] = {"value": r["value"], "unit": "Mvis/s", "ms_per_step": r["ms_per_step"],
                         "latency_ms": r["latency_ms"], "dtype": r["dtype"], "roofline": r["roofline"],
                         "stages_ms_per_launch": r["stages_ms_per_launch"], "config": r["config"],
                         "setup": r["setup"]}
    if not args.no_cpu_baseline and not planes:
        workers = args.cpu_workers or min(16, host_cores())
        log(f"CPU baseline on {workers} processes")
        result["cpu_baseline"] = cpu_baseline(wl, uvw, args.cpu_sample, workers)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
