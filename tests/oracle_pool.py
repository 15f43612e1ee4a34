"""Exact oracle kernels of many visibilities in parallel (test infrastructure).

Worker processes are spawned (not forked), so they never inherit a GPU
context; they import only the oracle and numpy/scipy.  Pool size follows the
host's CPU share, at most 16.
"""
from __future__ import annotations

import concurrent.futures as cf
import multiprocessing as mp
import os

from oracle import wkernel


def _kernel(args):
    u, v, w, geom, jp = args
    return wkernel.visibility_kernel(u, v, w, geom, jp)


def workers() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def fill_kernels(ref, idx, n_workers: int | None = None):
    """Compute ref.kernel(p) for every p in idx (exact Eq. (6) kernels) in parallel."""
    assert ref.kernel_fn is wkernel.visibility_kernel
    todo = sorted({int(p) for p in idx} - set(ref._kernels))
    if not todo:
        return
    n_workers = n_workers or workers()
    if n_workers <= 1 or len(todo) < 16:
        for p in todo:
            ref.kernel(p)
        return
    args = [(float(ref.u_pix[p]), float(ref.v_pix[p]), float(ref.w_eff[p]), ref.geom, int(ref.jp[p]))
            for p in todo]
    # costliest first, so the pool ends evenly
    order = sorted(range(len(todo)), key=lambda i: -args[i][4])
    with cf.ProcessPoolExecutor(n_workers, mp_context=mp.get_context("spawn")) as ex:
        results = ex.map(_kernel, [args[i] for i in order], chunksize=1)
        for i, res in zip(order, results):
            ref._kernels[todo[i]] = res
