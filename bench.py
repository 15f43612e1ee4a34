"""Benchmark: degrid + grid throughput with per-visibility exact w-kernels.

One step is one application of the measurement operator and its adjoint
(y = Phi x, then x' = Re Phi^dagger y) over all visibilities, with the
kernels already built and resident in HBM (the metric's definition).
Folding, k-means, sorting and the kernel build run once before the timed
region and are reported separately.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Prints one JSON line.  Inputs are seeded synthetic MWA-like data (the
paper's Fornax A visibilities are not available).
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
    ap.add_argument("--workload", default="mwa_1024_single_stack")
    ap.add_argument("--precision", default=None, help="override: fp32_fp64phase or fp64")
    ap.add_argument("--m-vis", type=int, default=None, help="override visibility count (debug)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=2000)
    ap.add_argument("--stacks", type=int, default=None, help="override the workload's w-stack count")
    ap.add_argument("--fold", type=int, choices=[0, 1], default=None,
                    help="override the workload's conjugate-symmetry folding")
    ap.add_argument("--kernels", default="exact", choices=["exact", "planes"],
                    help="exact per-visibility taps, or taps interpolated from 1-D w-planes")
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


def algorithmic_bytes(stage: str, taps: int, m: int, cells: int, cb: int) -> int:
    """Bytes one launch must move at minimum.

    degrid: every tap once, the grid cells once, per visibility its base
    (8 B), weight (4 B) and output (cb B).  grid: the same with the
    visibility read instead of written and the grid written once.
    """
    per_vis = 8 + 4 + cb
    return taps * cb + m * per_vis + cells * cb


# w-plane mode: FP32 operations per tap of the interpolation and the
# multiply-add, counting an FMA as two (distance 6, lattice index 3, bilinear
# complex interpolation 18, conjugation 1, complex multiply-add 8)
PLANE_FLOPS_PER_TAP = 36
# VALU FP32 peak without packed FP32 instructions (not used by this build):
# 256 CUs x 64 lanes x 2 (FMA) x 2.4 GHz
VALU_FP32_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12


def cpu_baseline(wl, uvw, x, y, sample_n: int):
    """Time the FP64 oracle's degrid + grid on a bounded sample and scale to M.

    The sample is ``sample_n`` visibilities at uniform quantiles of J_p, so
    its mean cost per visibility estimates the workload's.  As on the GPU,
    kernel construction is outside the step: the oracle's kernel cache is
    filled with seeded random taps of each visibility's true shape (its
    degrid / grid cost depends only on the shapes).  Each timing is the
    minimum of three runs; the fixed part (FFTs, taper, crop) is timed with a
    single visibility per stack.
    """
    from oracle import operator, wkernel
    geom = wkernel.Geometry(n=wl.n, fov=math.radians(wl.fov_deg))
    ref = operator.StackedOperator(geom, uvw, n_stacks=wl.n_stacks, fold=wl.fold)
    m = ref.m
    order = np.argsort(ref.jp, kind="stable")
    sample = np.unique(order[np.linspace(0, m - 1, min(sample_n, m)).astype(np.int64)])
    rng = np.random.default_rng(11)
    for p in sample:
        jp = int(ref.jp[p])
        u0, v0, _ = wkernel.tap_geometry(ref.u_pix[p], ref.v_pix[p], jp)
        ref._kernels[int(p)] = (u0, v0, rng.normal(size=(jp, jp)) + 1j * rng.normal(size=(jp, jp)))
    # one visibility of each stack present in the sample: the fixed part per stack
    firsts = np.array([sample[ref.labels[sample] == k][0] for k in range(ref.n_stacks)
                       if np.any(ref.labels[sample] == k)])

    def best(f, reps=3):
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            f()
            t.append(time.perf_counter() - t0)
        return min(t)

    t_fwd = best(lambda: ref.forward(x, subset=sample))
    t_adj = best(lambda: ref.adjoint(y, subset=sample))
    t_fwd1 = best(lambda: ref.forward(x, subset=firsts))
    t_adj1 = best(lambda: ref.adjoint(y, subset=firsts))
    n_s, n_1 = len(sample), len(firsts)
    per_vis = max((t_fwd - t_fwd1) + (t_adj - t_adj1), 0.0) / max(n_s - n_1, 1)
    fixed = (t_fwd1 + t_adj1) * ref.n_stacks / n_1
    t_step = fixed + per_vis * m
    return {
        "value": m / t_step / 1e6,
        "unit": "Mvis/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{n_s} visibilities at uniform J_p quantiles (J_p {int(ref.jp[sample].min())}-"
                   f"{int(ref.jp[sample].max())}); oracle degrid + grid, min of 3 runs, mean cost "
                   f"per visibility scaled to all {m}, plus the per-stack FFT / taper / crop part "
                   f"timed with one visibility per stack; kernel construction excluded (random "
                   f"taps of the true shapes in the oracle's kernel cache)"),
        "per_vis_us": per_vis * 1e6,
        "fixed_s": fixed,
        "extrapolated_step_s": t_step,
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
    """Continuous-batching server fed by a seeded Poisson stream (see serving.py)."""
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
    srv = Server(hbm_budget=int(args.serve_budget_gb * 2**30))
    t0 = time.perf_counter()
    refused = []
    for name, n, m, k, fold in specs:
        params = wsp.make_params(n, math.radians(25.0), n_stacks=k, fold=fold)
        try:
            srv.register_job(name, params, base[:m])
        except ValueError:
            refused.append(name)
        log(f"registered {name}: N={n} M={m} K={k} ({time.perf_counter() - t0:.1f} s)")
    if srv.waiting_jobs:
        raise RuntimeError("jobs left waiting at start; raise --serve-budget-gb")
    live = [s for s in specs if s[0] not in refused]
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
    for r in reqs:
        r.result = None
    # saturated: the same requests all queued at once (closed loop); requests of
    # different jobs run concurrently, each job's in order
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
    for r in sat:
        r.result = None
    log(f"saturated: {len(sat)} requests in {wall_sat:.2f} s")
    for name in list(srv.jobs):
        if srv.jobs[name].op is not None:
            srv.retire_job(name)
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
        log(f"fp64 baseline {name} done")
    unbatched64_s = sum(t64[(r.job_id, r.kind)] for r in reqs)
    print(json.dumps({
        "metric": "served operator requests: p50/p99 latency and Mvis/s",
        "mode": "serving", "requests": len(reqs), "wall_s": wall,
        "value": vis / wall / 1e6, "unit": "Mvis/s",
        "latency_ms": lat, "offered_load": args.serve_load,
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

    import torch

    from paper_1903_06555_amd import synthetic as syn
    from paper_1903_06555_amd import wsp

    wl = syn.WORKLOADS[args.workload]
    precision = args.precision or wl.precision
    m = args.m_vis or wl.m_vis
    uvw = syn.workload_uvw(wl, m)
    x_np = syn.workload_sky(wl)
    dev = torch.device("cuda", 0)
    fp64 = precision == "fp64"
    rdt = torch.float64 if fp64 else torch.float32
    cdt = torch.complex128 if fp64 else torch.complex64
    cb = 16 if fp64 else 8

    planes = args.kernels == "planes"
    params = wsp.make_params(wl.n, math.radians(wl.fov_deg), n_stacks=wl.n_stacks, fold=wl.fold,
                             precision=precision, kernels=args.kernels)
    t0 = time.perf_counter()
    op = wsp.Operator(params, uvw, build=False)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    log(f"plan done in {t_plan:.1f} s ({m} visibilities)")
    t0 = time.perf_counter()
    op.build(part=max(1, m // 10),
             progress=lambda d, n: log(f"built {d}/{n} kernels, {time.perf_counter() - t0:.1f} s"))
    t_build = time.perf_counter() - t0
    panels, capped = op.quad_stats()
    jp, _ = op.support()
    taps = int(np.sum(jp.astype(np.int64) ** 2))
    G = int(round(params.oversample * wl.n))
    cells = G * G * wl.n_stacks

    x = torch.from_numpy(x_np).to(dev, rdt)
    y = torch.empty(m, dtype=cdt, device=dev)
    xo = torch.empty((wl.n, wl.n), dtype=rdt, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        op.degrid(x, out=y)
        op.grid(y, out=xo)
    torch.cuda.synchronize()

    log("warmup done")
    wsp.wsp_set_timing(op.ctx, True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        op.degrid(x, out=y)
        op.grid(y, out=xo)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stages = wsp.wsp_stage_times(op.ctx)
    wsp.wsp_set_timing(op.ctx, False)
    lat = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
    ms_per_step = wall * 1e3 / args.steps

    per_launch = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in stages.items()}
    dom = "degrid" if per_launch["degrid"] >= per_launch["grid"] else "grid"
    if planes:
        flops = PLANE_FLOPS_PER_TAP * taps
        achieved_t = flops / (per_launch[dom] * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": dom, "achieved": achieved_t, "peak": VALU_FP32_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": achieved_t / VALU_FP32_PEAK_TFLOPS,
                    "traffic": measured_traffic(dom, wl.name + "_planes", m, precision),
                    "algorithmic_flops": flops, "flops_per_tap": PLANE_FLOPS_PER_TAP,
                    "lattice_bytes": op.footprint["kernel_bytes"], "avg_launch_ms": per_launch[dom]}
    else:
        traffic = algorithmic_bytes(dom, taps, m, cells, cb)
        achieved = traffic / (per_launch[dom] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "traffic": measured_traffic(dom, wl.name, m, precision),
                    "algorithmic_bytes": traffic, "avg_launch_ms": per_launch[dom]}

    y_host = y.cpu().numpy().astype(np.complex128)
    result = {
        "metric": ("Mvis/s degrid+grid with w-kernels interpolated on the fly from 1-D w-planes; "
                   "p50/p99 operator latency" if planes else
                   "Mvis/s degrid+grid with per-vis exact w-kernels; p50/p99 operator latency"),
        "value": m / (ms_per_step * 1e-3) / 1e6,
        "unit": "Mvis/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if fp64 else "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "fov_deg": wl.fov_deg, "m_vis": m,
                   "n_stacks": wl.n_stacks, "fold": wl.fold, "precision": precision,
                   "oversample": params.oversample, "kb_support": params.kb_support,
                   **({"kernels": "planes", "plane_dq": 1 / 64, "plane_dw": 1 / 16} if planes else {})},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "roofline": roofline,
        "stages_ms_per_launch": per_launch,
        "setup": {"plan_s": t_plan, "build_s": t_build, "build_mvis_per_s": m / t_build / 1e6,
                  "kernel_bytes": op.footprint["kernel_bytes"], "taps": taps,
                  "mean_jp": float(jp.mean()), "max_jp": int(jp.max()),
                  "quad_panels": panels, "quad_capped": capped},
    }
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step")
    if not args.no_cpu_baseline:
        yr = y_host
        result["cpu_baseline"] = cpu_baseline(wl, uvw, x_np, yr, args.cpu_sample)
    op.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
