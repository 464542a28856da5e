"""Seeded input generators: determinism, exact sizes and structure."""
import os
import subprocess
import sys

import numpy as np
import pytest

import graphgen


def test_splitmix64_known_values():
    # SplitMix64 seeded with 0: the first outputs of the reference generator
    # (state += 0x9e3779b97f4a7c15, then the mix) are published constants.
    g = 0x9E3779B97F4A7C15
    outs = [graphgen.mix64((k + 1) * g) for k in range(3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_er_exact_and_simple():
    n, m = 1000, 4000
    s, d = graphgen.er(n, m, 3)
    assert s.size == m and s.dtype == np.int32
    assert np.all(s != d)
    assert s.min() >= 0 and max(s.max(), d.max()) < n
    key = np.minimum(s, d).astype(np.int64) * n + np.maximum(s, d)
    assert np.unique(key).size == m
    s2, d2 = graphgen.er(n, m, 3)
    assert np.array_equal(s, s2) and np.array_equal(d, d2)
    s3, _ = graphgen.er(n, m, 4)
    assert not np.array_equal(s, s3)


def test_er_rejects_too_many_edges():
    with pytest.raises(ValueError):
        graphgen.er(4, 7, 1)


def test_grid_counts_and_structure():
    rows, cols = 40, 50
    total = graphgen.lattice_edges(rows, cols)
    assert total == 2 * rows * cols - rows - cols
    s, d = graphgen.grid_holes(rows, cols, 0.1, 2)
    assert s.size == total - round(0.1 * total)
    assert np.all(s < d)
    diff = d - s
    assert np.all((diff == 1) | (diff == cols))
    assert np.all((diff != 1) | (s % cols != cols - 1))
    key = s.astype(np.int64) * rows * cols + d
    assert np.unique(key).size == s.size


def test_grid_full_size_count():
    assert graphgen.lattice_edges(4096, 4096) == 33546240
    assert 33546240 - round(0.1 * 33546240) == 30191616


def test_grid_permuted_is_relabelling():
    s, d = graphgen.grid_holes(30, 30, 0.2, 5, permute_ids=False)
    ps, pd = graphgen.grid_holes(30, 30, 0.2, 5, permute_ids=True)
    perm = graphgen.permutation(900, 5)
    a, b = perm[s], perm[d]
    assert np.array_equal(np.minimum(a, b), ps) and np.array_equal(np.maximum(a, b), pd)


def test_partial_lattice_for_batches():
    # first nv row-major vertices of a rows x cols grid
    assert graphgen.lattice_edges(3, 4, 10) == 7 + 6   # horizontal 3+3+1, vertical 6


def test_permutation_is_bijection():
    p = graphgen.permutation(10000, 9)
    assert np.array_equal(np.sort(p), np.arange(10000))


def test_rmat_shape_and_skew():
    s, d = graphgen.rmat(12, 8, 1, permute_ids=False)
    assert s.size == 8 << 12
    assert s.min() >= 0 and max(s.max(), d.max()) < 4096
    # without the permutation, quadrant a = 0.57 puts vertex 0 as the top hub
    deg = np.bincount(np.concatenate([s, d]), minlength=4096)
    assert deg.argmax() == 0
    # P(top bit of src set) = c + d = 0.24
    frac = np.mean(s >= 2048)
    assert abs(frac - 0.24) < 0.01


def test_rmat_thread_count_independent(tmp_path):
    code = ("import graphgen, numpy as np, sys; s, d = graphgen.rmat(14, 4, 7);"
            "np.save(sys.argv[1], np.stack([s, d]))")
    out = []
    for t in ("1", "3"):
        f = str(tmp_path / ("r%s.npy" % t))
        env = dict(os.environ, OMP_NUM_THREADS=t)
        subprocess.check_call([sys.executable, "-c", code, f], env=env,
                              cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
        out.append(np.load(f))
    assert np.array_equal(out[0], out[1])


def test_batch_distribution():
    b = graphgen.batch(3000, 1)
    assert b.n.min() >= 64 and b.n.max() <= 1 << 20
    med = np.median(b.n)
    assert 1700 < med < 2300
    assert 0.4 < b.kind.mean() < 0.6
    assert b.edge_off[-1] == b.m.sum() and b.vertex_off[-1] == b.n.sum()
    for g in range(0, 3000, 97):
        s, d, n = b.graph(g)
        assert s.size == b.m[g]
        if s.size:
            assert s.min() >= 0 and max(s.max(), d.max()) < n
        if b.kind[g] == 0:
            assert np.all(s != d)


def test_poisson_trace():
    t, big, pick = graphgen.poisson_trace(20000, 2000.0, 0.01, 500, 8, 3)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] - 10.0) < 0.5
    assert 100 < big.sum() < 320
    assert pick[big == 1].max() < 8 and pick[big == 0].max() < 500
