"""Pins of the CPU oracle against things other than itself.

The oracle's result is the plain definition "minimum vertex id of the
component" (Section II-A, Theorem "Graph Convergence").  It is pinned by:
  * hand-worked golden cases (tests/golden/tiny_graphs.txt);
  * exhaustive comparison with a reachability closure (Warshall) over every
    labelled graph with n <= 6;
  * BFS and scipy's connected_components as independent routes on random and
    full-size graphs;
  * the invariants of a converged label array (one star per component whose
    root is its minimum);
  * planted mistakes: mutated copies of the oracle's C source must fail these
    pins (the mutation test at the end).
"""
import itertools
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_tiny():
    cases = []
    with open(os.path.join(GOLDEN, "tiny_graphs.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            name, n, edges, labels = [p.strip() for p in line.split("|")]
            n = int(n)
            pairs = [tuple(int(x) for x in e.split("-")) for e in edges.split()]
            src = np.array([p[0] for p in pairs], np.int32)
            dst = np.array([p[1] for p in pairs], np.int32)
            exp = np.array([int(x) for x in labels.split()], np.int32)
            cases.append((name, n, src, dst, exp))
    return cases


TINY = load_tiny()


@pytest.mark.parametrize("case", TINY, ids=[c[0] for c in TINY])
def test_golden_tiny(case):
    name, n, src, dst, exp = case
    assert np.array_equal(oracle.uf_labels(src, dst, n), exp)
    assert np.array_equal(oracle.bfs_labels(src, dst, n), exp)


def closure_labels(n, pairs):
    """Minimum reachable id from a boolean reachability closure (Warshall)."""
    r = np.eye(n, dtype=bool)
    for a, b in pairs:
        r[a, b] = r[b, a] = True
    for k in range(n):
        r |= r[:, [k]] & r[[k], :]
    return np.array([np.flatnonzero(r[v])[0] for v in range(n)], np.int32)


def all_graphs(n):
    slots = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(slots)):
        yield [slots[i] for i in range(len(slots)) if mask >> i & 1]


def test_exhaustive_small_graphs_n_le_5():
    count = 0
    for n in range(0, 6):
        for pairs in all_graphs(n):
            src = np.array([p[0] for p in pairs], np.int32)
            dst = np.array([p[1] for p in pairs], np.int32)
            exp = closure_labels(n, pairs) if n else np.empty(0, np.int32)
            assert np.array_equal(oracle.uf_labels(src, dst, n), exp), (n, pairs)
            assert np.array_equal(oracle.uf_labels(dst, src, n), exp), (n, pairs)
            assert np.array_equal(oracle.bfs_labels(src, dst, n), exp), (n, pairs)
            count += 1
    assert count == 1 + 1 + 2 + 8 + 64 + 1024


def test_exhaustive_n6_with_reversed_edge_order():
    n = 6
    for pairs in all_graphs(n):
        exp = closure_labels(n, pairs)
        src = np.array([p[1] for p in pairs][::-1], np.int32)
        dst = np.array([p[0] for p in pairs][::-1], np.int32)
        assert np.array_equal(oracle.uf_labels(src, dst, n), exp), pairs


@pytest.mark.parametrize("n,m,seed", [(64, 20, 1), (64, 64, 2), (1000, 300, 3), (1000, 500, 4),
                                      (1000, 1000, 5), (5000, 20000, 6), (65536, 16384, 7),
                                      (65536, 32768, 8), (65536, 65536, 9)])
def test_random_er_three_routes(n, m, seed):
    src, dst = graphgen.er(n, m, seed)
    a = oracle.uf_labels(src, dst, n)
    assert np.array_equal(a, oracle.bfs_labels(src, dst, n))
    assert np.array_equal(a, oracle.scipy_labels(src, dst, n))
    ncomp = np.unique(a).size
    assert oracle.check_labels(src, dst, n, a, ncomp) == []


def test_er_config_full_size():
    n, m = 65536, 524288
    src, dst = graphgen.er(n, m, 1)
    a = oracle.uf_labels(src, dst, n)
    assert np.array_equal(a, oracle.scipy_labels(src, dst, n))
    assert oracle.check_labels(src, dst, n, a) == []


@pytest.mark.parametrize("permute", [False, True])
def test_grid_with_holes_three_routes(permute):
    src, dst = graphgen.grid_holes(256, 256, 0.1, 3, permute_ids=permute)
    n = 256 * 256
    a = oracle.uf_labels(src, dst, n)
    assert np.array_equal(a, oracle.bfs_labels(src, dst, n))
    assert np.array_equal(a, oracle.scipy_labels(src, dst, n))
    assert np.unique(a).size > 1


def test_rmat_three_routes():
    src, dst = graphgen.rmat(14, 4, 5)
    n = 1 << 14
    a = oracle.uf_labels(src, dst, n)
    assert np.array_equal(a, oracle.bfs_labels(src, dst, n))
    assert np.array_equal(a, oracle.scipy_labels(src, dst, n))


def test_batch_oracle_matches_per_graph():
    b = graphgen.batch(40, 11, median=200, n_hi=5000)
    lab = oracle.uf_batch(b.edge_off, b.vertex_off, b.src, b.dst)
    for g in range(b.num_graphs):
        s, d, n = b.graph(g)
        v0 = int(b.vertex_off[g])
        assert np.array_equal(lab[v0:v0 + n], oracle.scipy_labels(s, d, n))


def test_rejects_out_of_range_ids():
    with pytest.raises(ValueError):
        oracle.uf_labels(np.array([0, 3], np.int32), np.array([1, 1], np.int32), 3)
    with pytest.raises(ValueError):
        oracle.uf_labels(np.array([-1], np.int32), np.array([0], np.int32), 3)
    with pytest.raises(ValueError):
        oracle.bfs_labels(np.array([0], np.int32), np.array([5], np.int32), 5)


def test_invariant_checker_catches_violations():
    src = np.array([0, 1, 3], np.int32)
    dst = np.array([1, 2, 4], np.int32)
    good = np.array([0, 0, 0, 3, 3], np.int32)
    assert oracle.check_labels(src, dst, 5, good, 2) == []
    assert oracle.check_labels(src, dst, 5, np.array([0, 0, 1, 3, 3], np.int32))  # edge split
    assert oracle.check_labels(src, dst, 5, np.array([1, 1, 1, 3, 3], np.int32))  # L[v] > v
    assert oracle.check_labels(src, dst, 5, good, 3)                              # root count


def test_diameter_lower_bound_on_lattice():
    # hole-free rows x cols lattice: diameter rows + cols - 2 (corner to corner)
    src, dst = graphgen.grid_holes(20, 30, 0.0, 1)
    assert oracle.diameter_lower_bound(src, dst, 600, 0) == 48


# ---------------------------------------------------------- planted bugs --

MUTANTS = {
    # larger root linked under... the larger one: roots stop being minima
    "link_wrong_way": ("if (ru < rv) labels[rv] = ru;", "if (ru > rv) labels[rv] = ru;"),
    # final labels are parents instead of roots
    "no_final_find": ("for (int32_t i = 0; i < n; ++i) labels[i] = uf_find(labels, i);",
                      "for (int32_t i = 0; i < n; ++i) labels[i] = labels[i];"),
    # one endpoint used without find
    "skip_find_dst": ("int32_t rv = uf_find(labels, dst[e]);", "int32_t rv = dst[e];"),
    # last edge dropped
    "drop_last_edge": ("for (int64_t e = 0; e < m; ++e) {\n        int32_t ru",
                       "for (int64_t e = 0; e + 1 < m; ++e) {\n        int32_t ru"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_oracle_mistakes_are_caught(name, tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    text = open(os.path.join(os.path.dirname(oracle.__file__), "cc_oracle.c")).read()
    old, new = MUTANTS[name]
    assert old in text, "mutation anchor missing"
    src_path = tmp_path / "mutant.c"
    src_path.write_text(text.replace(old, new, 1))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-o", str(so), str(src_path)])
    import ctypes
    lib = ctypes.CDLL(str(so))
    p32 = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_uf_labels.argtypes = [p32, p32, ctypes.c_int64, ctypes.c_int32, p32]

    def mutant(src, dst, n):
        src = np.ascontiguousarray(src, np.int32)
        dst = np.ascontiguousarray(dst, np.int32)
        out = np.empty(n, np.int32)
        lib.oracle_uf_labels(src.ctypes.data_as(p32), dst.ctypes.data_as(p32), src.size, n,
                             out.ctypes.data_as(p32))
        return out

    caught = False
    for case in TINY:
        _, n, s, d, exp = case
        if n and not np.array_equal(mutant(s, d, n), exp):
            caught = True
    for n in range(2, 6):
        for pairs in all_graphs(n):
            s = np.array([p[1] for p in pairs], np.int32)
            d = np.array([p[0] for p in pairs], np.int32)
            if not np.array_equal(mutant(s, d, n), closure_labels(n, pairs)):
                caught = True
                break
    assert caught, "planted mistake %s went unnoticed" % name
