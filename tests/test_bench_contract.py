"""Host-side checks of the benchmark contract and the synthetic inputs (no GPU)."""
import json
import os
import subprocess
import sys

import numpy as np

from paper_1903_06555_amd import synthetic as syn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in json.loads(res.stdout.strip().splitlines()[-1])["error"]


def test_mwa_track_shape_and_w_range():
    uvw = syn.mwa_rotation_uvw(20000, 120.0)
    assert uvw.shape == (20000, 3)
    assert 400 < np.max(np.abs(uvw[:, 2])) < 520          # |w| up to ~500 wavelengths
    assert np.max(np.hypot(uvw[:, 0], uvw[:, 1])) < 3100   # 6 km max baseline at 2 m


def test_generators_are_seeded():
    a = syn.workload_uvw(syn.WORKLOADS["tiny_box_64"])
    b = syn.workload_uvw(syn.WORKLOADS["tiny_box_64"])
    assert np.array_equal(a, b)
    assert np.array_equal(syn.random_vis(10, 3), syn.random_vis(10, 3))
    x = syn.point_source_sky(64, 20, "gaussian", 1)
    assert np.count_nonzero(x) <= 20 and x.shape == (64, 64)


def test_traffic_record_matches_sources_workload_and_precision():
    import bench
    rec = bench.measured_traffic("grid", "mwa_1024_single_stack", 1_000_000, "fp32_fp64phase")
    assert rec is None or rec > 0
    # another precision, visibility count or workload never borrows that record
    assert bench.measured_traffic("grid", "mwa_1024_single_stack", 1_000_000, "fp64") is None
    assert bench.measured_traffic("grid", "mwa_1024_single_stack", 999_999, "fp32_fp64phase") is None
    assert bench.measured_traffic("grid", "no_such_workload", 1_000_000, "fp32_fp64phase") is None
