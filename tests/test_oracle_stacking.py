"""Pins for oracle.stacking: Algorithm 1 (k-means w-stacking) and Eq. (8) folding."""
import itertools

import numpy as np

from oracle import stacking


def test_hand_worked_two_stack_example():
    # init [0, 11] -> labels [0,0,1,1] -> centres [0.5, 10.5]; the second pass
    # changes nothing, so the relative change is 0 and the loop stops at t = 2.
    labels, centres, it = stacking.kmeans_w(np.array([0.0, 1.0, 10.0, 11.0]), 2)
    assert labels.tolist() == [0, 0, 1, 1]
    assert centres.tolist() == [0.5, 10.5]
    assert it == 2


def test_single_stack_is_the_mean():
    w = np.array([3.0, -1.0, 7.5, 2.25])
    labels, centres, it = stacking.kmeans_w(w, 1)
    assert labels.tolist() == [0, 0, 0, 0]
    assert centres[0] == np.mean(w)


def test_empty_stack_gets_zero_centre():
    labels, centres, it = stacking.kmeans_w(np.array([5.0, 5.0, 5.0, 6.0]), 3)
    assert labels.tolist() == [0, 0, 0, 2]
    assert centres.tolist() == [5.0, 0.0, 6.0]
    assert it == 2


def test_ties_go_to_lowest_stack():
    lab = stacking.assign(np.array([1.0, 2.0, 3.0]), np.array([1.0, 3.0]))
    assert lab.tolist() == [0, 0, 1]


def _is_lloyd_fixed_point(w, labels, k):
    centres, counts = stacking.update(w, labels, k)
    return np.array_equal(stacking.assign(w, centres), labels), centres


def test_result_is_a_brute_force_lloyd_fixed_point():
    rng = np.random.default_rng(3)
    k = 3
    for trial in range(4):
        w = np.round(rng.uniform(0, 100, 8), 3)
        labels, centres, _ = stacking.kmeans_w(w, k, tol=0.0, max_iter=500)
        fixed = set()
        for lab in itertools.product(range(k), repeat=w.size):
            lab = np.array(lab)
            ok, _ = _is_lloyd_fixed_point(w, lab, k)
            if ok:
                fixed.add(tuple(lab.tolist()))
        assert tuple(labels.tolist()) in fixed
        ok, c = _is_lloyd_fixed_point(w, labels, k)
        assert ok and np.array_equal(c, centres)


def test_within_stack_sse_is_monotone():
    rng = np.random.default_rng(4)
    w = np.concatenate([rng.normal(20, 5, 300), rng.normal(200, 30, 500), rng.uniform(0, 600, 200)])
    prev = np.inf
    for t in range(1, 25):
        labels, centres, it = stacking.kmeans_w(w, 6, tol=0.0, max_iter=t)
        sse = stacking.within_stack_sse(w, labels, centres)
        assert sse <= prev * (1 + 1e-12)
        prev = sse


def test_fold_is_strict_and_exact():
    uvw = np.array([[1.0, 2.0, -3.0], [4.0, -5.0, 0.0], [-7.0, 8.0, 9.0], [0.5, 0.25, -0.0]])
    out, flag = stacking.fold(uvw)
    assert flag.tolist() == [True, False, False, False]
    assert out[0].tolist() == [-1.0, -2.0, 3.0]
    assert np.array_equal(out[1:], uvw[1:])
