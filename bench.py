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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mwa_1024_single_stack")
    ap.add_argument("--precision", default=None, help="override: fp32_fp64phase or fp64")
    ap.add_argument("--m-vis", type=int, default=None, help="override visibility count (debug)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=6)
    ap.add_argument("--mode", default="operator", choices=["operator", "copy"],
                    help="operator: the metric; copy: a plain 2 GiB device copy used to "
                         "calibrate rocprofv3 FETCH_SIZE / WRITE_SIZE readings")
    return ap.parse_args()


def algorithmic_bytes(stage: str, taps: int, m: int, cells: int, cb: int) -> int:
    """Bytes one launch must move at minimum (measurement).

    degrid: every tap once, the grid cells once, per visibility its base
    (8 B), weight (4 B) and output (cb B).  grid: the same with the
    visibility read instead of written and the grid written once.
    """
    per_vis = 8 + 4 + cb
    return taps * cb + m * per_vis + cells * cb


def cpu_baseline(wl, uvw, x, y, sample_n: int, total_taps: int, jp_all):
    """Time the FP64 oracle on a bounded sample and scale to the workload."""
    from oracle import operator, wkernel
    geom = wkernel.Geometry(n=wl.n, fov=math.radians(wl.fov_deg))
    ref = operator.StackedOperator(geom, uvw, n_stacks=wl.n_stacks, fold=wl.fold)
    order = np.argsort(ref.jp, kind="stable")
    qs = np.linspace(0.1, 0.9, sample_n)
    sample = np.unique(order[(qs * (len(order) - 1)).astype(int)])
    t0 = time.perf_counter()
    for p in sample:
        ref.kernel(int(p))            # kernels resident, as on the GPU (untimed below)
    t_build = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref.stack_grid(x, 0)
    t_fft_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref.forward(x, subset=sample)
    t_fwd = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref.adjoint(y, subset=sample[:1])
    t_adj1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref.adjoint(y, subset=sample)
    t_adj = time.perf_counter() - t0
    taps_sample = int(np.sum(ref.jp[sample].astype(np.int64) ** 2))
    taps_first = int(ref.jp[sample[0]]) ** 2
    per_tap = ((t_fwd - t_fft_fwd) + (t_adj - t_adj1)) / max(taps_sample - taps_first, 1) \
        if taps_sample > taps_first else (t_fwd - t_fft_fwd) / taps_sample
    per_tap = max(per_tap, 0.0)
    t_step = t_fft_fwd + t_adj1 + per_tap * total_taps
    m = uvw.shape[0]
    return {
        "value": m / t_step / 1e6,
        "unit": "Mvis/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{len(sample)} visibilities at J_p quantiles 0.1-0.9 (J_p {int(ref.jp[sample].min())}-"
                   f"{int(ref.jp[sample].max())}); oracle degrid+grid time per tap on the sample "
                   f"scaled to all {total_taps} taps, plus one full-size FFT pair; kernels "
                   f"built beforehand ({t_build:.1f} s, untimed)"),
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


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.mode == "copy":
        copy_calibration(args.steps)
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

    params = wsp.make_params(wl.n, math.radians(wl.fov_deg), n_stacks=wl.n_stacks, fold=wl.fold,
                             precision=precision)
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
    traffic = algorithmic_bytes(dom, taps, m, cells, cb)
    achieved = traffic / (per_launch[dom] * 1e-3) / 1e9

    y_host = y.cpu().numpy().astype(np.complex128)
    result = {
        "metric": "Mvis/s degrid+grid with per-vis exact w-kernels; p50/p99 operator latency",
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
                   "oversample": params.oversample, "kb_support": params.kb_support},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes": traffic, "avg_launch_ms": per_launch[dom]},
        "stages_ms_per_launch": per_launch,
        "setup": {"plan_s": t_plan, "build_s": t_build, "build_mvis_per_s": m / t_build / 1e6,
                  "kernel_bytes": op.footprint["kernel_bytes"], "taps": taps,
                  "mean_jp": float(jp.mean()), "max_jp": int(jp.max()),
                  "quad_panels": panels, "quad_capped": capped},
    }
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step")
    if not args.no_cpu_baseline:
        yr = y_host
        result["cpu_baseline"] = cpu_baseline(wl, uvw, x_np, yr, args.cpu_sample, taps, jp)
    op.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
