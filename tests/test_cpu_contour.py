"""The paper's multicore CPU design (oracle/contour_omp.c): asynchronous
update, early convergence check and plain stores on all host threads
(Algorithm 1, Section III-B).  It is the timed CPU Contour baseline of the
benchmark, so its labels must equal the union-find oracle's on every family
and order; sweep counts depend on the thread interleaving and are only
bounded."""
import numpy as np
import pytest

import graphgen
import oracle


@pytest.mark.parametrize("order", [1, 2, 3, 0])
def test_contour_omp_equals_union_find(order):
    cases = [(graphgen.er(1000, 1500, 1), 1000), (graphgen.er(5000, 2000, 2), 5000),
             (graphgen.grid_holes(120, 90, 0.1, 3, permute_ids=True), 120 * 90),
             (graphgen.rmat(14, 8, 4), 1 << 14)]
    for (src, dst), n in cases:
        lab, sweeps, threads = oracle.contour_omp(src, dst, n, order)
        assert np.array_equal(lab, oracle.uf_labels(src, dst, n)), (n, order)
        assert threads >= 1 and sweeps >= 2


def test_contour_omp_degenerate_inputs():
    e = np.zeros(0, np.int32)
    lab, sweeps, _ = oracle.contour_omp(e, e, 5)
    assert np.array_equal(lab, np.arange(5)) and sweeps == 0
    lab, _, _ = oracle.contour_omp(np.array([2, 2]), np.array([2, 0]), 3)
    assert np.array_equal(lab, [0, 1, 0])
    with pytest.raises(ValueError):
        oracle.contour_omp(np.array([0]), np.array([3]), 3)


def test_contour_omp_path_sweeps_within_order1_bound():
    # order 1 on the increasing path: one sweep per hop at worst (the
    # synchronous count n - 1 changing sweeps), fewer when the in-place
    # update carries labels further within a sweep
    n = 300
    lab, sweeps, _ = oracle.contour_omp(np.arange(n - 1), np.arange(1, n), n, 1)
    assert np.all(lab == 0) and 2 <= sweeps <= n
