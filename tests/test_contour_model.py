"""Pins of the CPU models of the Contour algorithm (oracle/contour_model.py).

The models replay Definition 3 / Algorithm 1 and the asynchronous variant of
Section III-B.  They are pinned by closed forms derived by hand from
Definition 3 (tests/golden/closed_forms.txt), by the final labels of the
union-find and BFS oracles, and by the invariants of Section II-A.

Hand derivations (increasing-id path 0-1-...-(n-1), synchronous):
  order 1: the edge <j-1, j> gives L_u[j] = L[j-1]; from L[j] = j - k this is
           j - k - 1, so L[j] = max(0, j - k) after k iterations and n - 1
           iterations change something.
  order 2: with L[j] = j - d, edge <j-1, j> has L^2[j-1] = j - 1 - 2d, so the
           offset grows d -> 2d + 1, d_k = 2^k - 1 and ceil(log2 n) iterations
           change something.
  chase to root: iteration 1 sets L[j] = j - 1 (every vertex is a root, the
           larger one is hooked); iteration 2 follows each chain to 0 and maps
           every vertex to 0: 2 changing iterations for n >= 3.
"""
import itertools
import os
import random

import numpy as np
import pytest

import graphgen
import oracle
from oracle import contour_model as cm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def closed_form_cases():
    out = []
    with open(os.path.join(GOLDEN, "closed_forms.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            fam, n, order, changing = [p.strip() for p in line.split("|")]
            out.append((fam, int(n), int(order), int(changing)))
    return out


def family(fam, n):
    if fam == "path":
        return np.arange(n - 1), np.arange(1, n)
    if fam == "complete":
        pairs = list(itertools.combinations(range(n), 2))
        return np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs])
    raise ValueError(fam)


@pytest.mark.parametrize("case", closed_form_cases(), ids=lambda c: "%s-n%d-h%d" % c[:3])
def test_sync_closed_forms(case):
    fam, n, order, changing = case
    src, dst = family(fam, n)
    labels, iters, chg, _ = cm.contour_sync(src, dst, n, order)
    assert chg == changing
    assert iters == changing + 1
    assert np.all(labels == 0)


def test_sync_path_order1_states_follow_closed_form():
    n = 12
    src, dst = family("path", n)
    _, _, _, states = cm.contour_sync(src, dst, n, 1, record=True)
    for k, L in enumerate(states, start=1):
        assert np.array_equal(L, np.maximum(0, np.arange(n) - k))


def test_sync_path_order2_states_follow_closed_form():
    n = 40
    src, dst = family("path", n)
    _, _, _, states = cm.contour_sync(src, dst, n, 2, record=True)
    for k, L in enumerate(states, start=1):
        assert np.array_equal(L, np.maximum(0, np.arange(n) - (2 ** k - 1)))


def all_graphs(n):
    slots = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(slots)):
        yield [slots[i] for i in range(len(slots)) if mask >> i & 1]


@pytest.mark.parametrize("order", [1, 2, 3, cm.FULL])
def test_sync_exhaustive_n_le_5(order):
    for n in range(1, 6):
        for pairs in all_graphs(n):
            src = np.array([p[1] for p in pairs], np.int64)
            dst = np.array([p[0] for p in pairs], np.int64)
            exp = oracle.bfs_labels(src, dst, n)
            assert np.array_equal(cm.contour_sync(src, dst, n, order)[0], exp), (order, pairs)


@pytest.mark.parametrize("name", ["C-1", "C-2", "C-m", "C-11mm", "C-1m1m", "C-full", "C-3"])
def test_sync_and_async_schedules_reach_oracle_labels(name):
    rng = random.Random(7)
    for trial in range(25):
        n = rng.randint(1, 60)
        m = rng.randint(0, min(2 * n, n * (n - 1) // 2))
        src, dst = graphgen.er(n, m, 100 + trial) if m else (np.zeros(0, np.int32),) * 2
        exp = oracle.uf_labels(src, dst, n)
        sched = cm.schedule(name)
        assert np.array_equal(cm.contour_sync(src, dst, n, sched)[0], exp)
        order = list(range(m))
        rng.shuffle(order)
        assert np.array_equal(cm.contour_async(src, dst, n, sched, order)[0], exp)


def test_async_never_needs_more_sweeps_than_order1_on_paths():
    # ordering of Section IV-C: iterations(C-m) <= iterations(C-2) <= iterations(C-1)
    for n in (10, 33, 100):
        src, dst = graphgen.grid_holes(1, n, 0.0, 1, permute_ids=True)
        s1 = cm.contour_sync(src, dst, n, 1)[1]
        s2 = cm.contour_sync(src, dst, n, 2)[1]
        sm = cm.contour_sync(src, dst, n, 1024)[1]
        assert sm <= s2 <= s1


def test_order_m_equals_chase_to_root_when_chains_are_short():
    src, dst = graphgen.er(200, 300, 3)
    a = cm.contour_sync(src, dst, 200, 1024, record=True)[3]
    b = cm.contour_sync(src, dst, 200, cm.FULL, record=True)[3]
    assert len(a) == len(b) and all(np.array_equal(x, y) for x, y in zip(a, b))


def test_theorem_bound_holds_for_sync_order2_on_small_graphs():
    # Graph Convergence theorem: at most ceil(log_{3/2} d_max) + 1 iterations
    # (here counted as changing iterations); checked on paths and grids.
    for n in (5, 17, 50, 200, 1000):
        src, dst = graphgen.grid_holes(1, n, 0.0, 2, permute_ids=True)
        chg = cm.contour_sync(src, dst, n, 2)[2]
        assert chg <= cm.theorem_bound(n - 1)
    for r, c in ((4, 4), (8, 8), (16, 16), (20, 30)):
        src, dst = graphgen.grid_holes(r, c, 0.0, 2)
        chg = cm.contour_sync(src, dst, r * c, 2)[2]
        assert chg <= cm.theorem_bound(r + c - 2)


def test_theorem_bound_values():
    assert cm.theorem_bound(1) == 1
    assert cm.theorem_bound(2) == 3          # ceil(1.709...) + 1
    assert cm.theorem_bound(8190) == 24
    assert cm.theorem_bound(11222) == 24     # 1.5**23 = 11222.7
    assert cm.theorem_bound(11223) == 25


def test_paper_check_equals_would_write_for_order2():
    # For order 2 the early convergence test of Section III-B-2 holds exactly
    # when the edge's conditional assignments would change something.
    rng = random.Random(3)
    for _ in range(3000):
        n = rng.randint(1, 9)
        # a random label array with L[x] <= x (a forest whose roots are minima)
        L = [rng.randint(0, x) for x in range(n)]
        w, v = rng.randrange(n), rng.randrange(n)
        _, values, z = cm.mm_edge_reads(L, w, v, 2)
        assert cm.paper_check(L, w, v) == any(val > z for val in values)


def test_lost_update_model_reaches_oracle_labels():
    rng = random.Random(5)
    for trial in range(60):
        n = rng.randint(2, 80)
        m = rng.randint(1, min(3 * n, n * (n - 1) // 2))
        src, dst = graphgen.er(n, m, 500 + trial)
        exp = oracle.uf_labels(src, dst, n)
        for order in (1, 2, 3, cm.FULL):
            lab, sweeps, ok = cm.contour_lost_update(src, dst, n, order, group=8, seed=trial)
            assert ok and np.array_equal(lab, exp), (trial, order)


def test_async_warm_start_from_partial_state():
    src, dst = graphgen.er(300, 400, 9)
    exp = oracle.uf_labels(src, dst, 300)
    _, _, _, states = cm.contour_sync(src, dst, 300, 2, record=True)
    mid = states[0]
    lab, _ = cm.contour_async(src, dst, 300, 2, L0=mid)
    assert np.array_equal(lab, exp)


def test_post_write_check_is_unsound():
    # Reading the early convergence check after an edge's own writes (instead
    # of on its pre-write reads) can stop before the fixed point; the model
    # uses pre-write reads.  A search over small random graphs finds a case
    # where the post-write reading ends with labels that differ from the oracle.
    rng = random.Random(11)
    found = False
    for trial in range(400):
        n = rng.randint(3, 10)
        m = rng.randint(1, n * (n - 1) // 2)
        src, dst = graphgen.er(n, m, 900 + trial)
        L = list(range(n))
        for _ in range(100):
            active = False
            for e in range(m):
                targets, _, z = cm.mm_edge_reads(L, int(src[e]), int(dst[e]), 2)
                for x in targets:
                    if L[x] > z:
                        L[x] = z
                if cm.paper_check(L, int(src[e]), int(dst[e])):
                    active = True
            if not active:
                break
        if not np.array_equal(np.array(L, np.int32), oracle.uf_labels(src, dst, n)):
            found = True
            break
    assert found


# ------------------------------------------------ sharded rounds (design) --

def _component_ids(src, dst, n):
    return oracle.uf_labels(src, dst, n)


@pytest.mark.parametrize("p", [1, 2, 4, 7])
@pytest.mark.parametrize("kind", ["er", "grid", "rmat"])
def test_sharded_rounds_reach_the_whole_graph_labels(kind, p):
    # the combine rule of the multi-GPU design: each round solves every
    # share from the current labels and keeps the elementwise minimum; the
    # run must end on the labels of the whole graph, with every round's
    # labels satisfying L[x] <= x, staying in x's component, never rising
    if kind == "er":
        src, dst = graphgen.er(300, 420, 3)
        n = 300
    elif kind == "grid":
        src, dst = graphgen.grid_holes(16, 20, 0.3, 4)
        n = 16 * 20
    else:
        src, dst = graphgen.rmat(8, 4, 5)
        n = 1 << 8
    share = np.random.default_rng(11 + p).integers(0, p, src.size)
    labels, rounds, states = cm.sharded_rounds(src, dst, n, share, p, record=True)
    exp = oracle.uf_labels(src, dst, n)
    assert np.array_equal(labels, exp)
    comp = _component_ids(src, dst, n)
    prev = np.arange(n)
    for L in states:
        assert (L <= np.arange(n)).all()
        assert np.array_equal(comp[L], comp)
        assert (L <= prev).all()
        prev = L
    if p == 1:
        assert rounds == 2  # one round solves, the next confirms
    assert rounds <= 64


def test_sharded_rounds_need_the_exchange():
    # a path split so that no share holds two consecutive edges: one round of
    # local solves cannot label the path, the exchange of minima must
    src = np.arange(0, 9, dtype=np.int32)
    dst = src + 1
    share = (np.arange(9) % 2).astype(np.int64)
    labels, rounds, states = cm.sharded_rounds(src, dst, 10, share, 2, record=True)
    assert np.array_equal(labels, np.zeros(10, np.int32))
    assert not np.array_equal(states[0], labels)
    assert rounds > 2


def test_sync_from_identity_equals_algorithm_1():
    src, dst = graphgen.er(200, 300, 9)
    a, it_a = cm.contour_sync_from(src, dst, np.arange(200), 2)
    b, it_b, _, _ = cm.contour_sync(src, dst, 200, 2)
    assert np.array_equal(a, b) and it_a == it_b


# ------------------------------------------------ incremental new edges --

@pytest.mark.parametrize("order", [1, 2, 3, cm.FULL])
@pytest.mark.parametrize("seed", range(12))
def test_add_edges_in_batches_reaches_whole_graph_labels(seed, order):
    # edges arrive in batches; after each batch only the new edges are swept
    # from the previous labels, then chains are flattened: the labels must be
    # those of every edge so far (the union-find oracle on the union)
    rng = np.random.default_rng(seed)
    kind = seed % 3
    if kind == 0:
        src, dst = graphgen.er(400, 500, seed)
        n = 400
    elif kind == 1:
        src, dst = graphgen.grid_holes(15, 25, 0.2, seed)
        n = 15 * 25
    else:
        src, dst = graphgen.rmat(8, 3, seed)
        n = 256
    cuts = np.sort(rng.integers(0, src.size + 1, 5))
    bounds = [0, *cuts.tolist(), src.size]
    L = np.arange(n, dtype=np.int32)
    for a, b in zip(bounds[:-1], bounds[1:]):
        L = cm.add_edges(L, src[a:b], dst[a:b], order)
        assert np.array_equal(L, oracle.uf_labels(src[:b], dst[:b], n))


def test_add_edges_needs_the_ties_to_old_roots():
    # Sweeping the new edges alone from the old labels is not enough: an
    # endpoint whose label is lowered stops pointing at its old root, and the
    # old edges that tie it to its component are not swept again.  With the
    # ties (x, old root of x) the whole-graph labels come out every time.
    src, dst = graphgen.er(400, 500, 0)
    old = oracle.uf_labels(src[:154], dst[:154], 400)
    bare = cm.flatten(cm.contour_sync_from(src[154:256], dst[154:256], old, 2)[0])
    assert not np.array_equal(bare, oracle.uf_labels(src[:256], dst[:256], 400))
    assert np.array_equal(cm.add_edges(old, src[154:256], dst[154:256], 2),
                          oracle.uf_labels(src[:256], dst[:256], 400))
    rng = np.random.default_rng(3)
    for trial in range(200):
        n = 12
        src, dst = graphgen.er(n, 8, trial)
        k = int(rng.integers(0, src.size + 1))
        L = cm.add_edges(oracle.uf_labels(src[:k], dst[:k], n), src[k:], dst[k:], 2)
        assert np.array_equal(L, oracle.uf_labels(src, dst, n)), trial


def test_flatten_of_a_chain():
    assert np.array_equal(cm.flatten([0, 0, 1, 2, 3, 5]), [0, 0, 0, 0, 0, 5])


# --------------------------------------------------- schedule closed forms --
# tests/golden/schedule_closed_forms.txt holds hand-derived iteration counts
# and per-iteration states of the operator schedules of Section III-B-4 on
# the increasing-id path (derivations in that file's header).

def schedule_cases():
    out = []
    with open(os.path.join(GOLDEN, "schedule_closed_forms.txt")) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            name, n, changing, states = [p.strip() for p in line.split("|")]
            out.append((name, int(n), int(changing), [int(d) for d in states.split(";")]))
    return out


def schedule_by_name(name):
    # the two variants that are not the paper's serve as planted mistakes:
    # a schedule that starts with order m, and C-11mm with k1 off by one
    if name == "C-m1m1":
        return lambda s: 1024 if s % 2 == 0 else 1
    if name.startswith("C-11mm-k1="):
        return cm.schedule("C-11mm", m=1024, k1=int(name.split("=")[1]))
    return cm.schedule(name, m=1024, k1=2)


@pytest.mark.parametrize("case", schedule_cases(), ids=lambda c: "%s-n%d" % c[:2])
def test_schedule_closed_forms_on_the_path(case):
    name, n, changing, offs = case
    src, dst = family("path", n)
    labels, iters, chg, states = cm.contour_sync(src, dst, n, schedule_by_name(name), record=True)
    assert chg == changing and iters == changing + 1
    assert np.all(labels == 0)
    for k, d in enumerate(offs):
        assert np.array_equal(states[k], np.maximum(0, np.arange(n) - d) if d else np.zeros(n)), (name, k)


def test_swapped_schedules_fail_the_closed_forms():
    # the closed forms tell the paper's schedules apart from their plausible
    # mistakes on n = 9: C-1m1m started with order m, C-11mm with k1 off by
    # one either way, and the two schedules swapped all change the count
    src, dst = family("path", 9)
    counts = {name: cm.contour_sync(src, dst, 9, schedule_by_name(name))[2]
              for name in ("C-11mm", "C-1m1m", "C-m1m1", "C-11mm-k1=1", "C-11mm-k1=3")}
    assert counts["C-1m1m"] == 2 and counts["C-m1m1"] == 3
    assert counts["C-11mm"] == 3 and counts["C-11mm-k1=1"] == 2 and counts["C-11mm-k1=3"] == 4
    assert counts["C-11mm"] != counts["C-1m1m"]


# ------------------------------------------------ asynchronous closed form --
# Section III-B-1: the update is in place, so a later edge of the same sweep
# reads what an earlier one stored.  Increasing-id path, order 1:
#   edges in increasing order <0,1>, <1,2>, ...: edge <j-1, j> reads
#   L[j-1] = 0 stored by the edge before it, so one sweep maps every vertex
#   to 0 (1 changing sweep, then one that changes nothing);
#   edges in decreasing order: edge <j-1, j> runs before <j-2, j-1> has
#   lowered L[j-1], so a sweep moves each label by one, exactly like the
#   synchronous update: n - 1 changing sweeps.
# A model that applied its stores to a copy (the synchronous update) would
# need n - 1 sweeps in both orders.

@pytest.mark.parametrize("n", [2, 3, 10, 57])
def test_async_in_place_closed_form_on_the_path(n):
    src, dst = family("path", n)
    inc = list(range(n - 1))
    lab, sweeps = cm.contour_async(src, dst, n, 1, inc)
    assert np.all(lab == 0) and sweeps == 2
    lab, sweeps = cm.contour_async(src, dst, n, 1, inc[::-1])
    assert np.all(lab == 0) and sweeps == (n - 1) + 1


# ----------------------------------------------------- lost-update pin ----
# Section III-B-3: plain stores may lose updates.  Vertices 0, 1, 2 with the
# edges <1, 2> and <0, 2> in one group, order 2, identity labels: edge <1, 2>
# reads z = 1 and stores L[2] = 1, edge <0, 2> reads z = 0 and stores
# L[2] = 0.  Applied in the order (L[2] = 0, L[2] = 1) the smaller value is
# overwritten, so L[2] = 1 after the first sweep; in the other order L[2] = 0.
# Either way the next sweeps reach the labels [0, 0, 0].  A model whose
# stores took the minimum (nothing lost) would always show L[2] = 0.

def test_lost_update_model_really_loses_stores():
    src, dst = np.array([1, 0]), np.array([2, 2])
    after_first = set()
    for seed in range(40):
        lab, sweeps, ok, states = cm.contour_lost_update(src, dst, 3, 2, group=8, seed=seed, record=True)
        assert ok and np.array_equal(lab, [0, 0, 0])
        after_first.add(int(states[0][2]))
        if states[0][2] == 1:
            # the lost store costs a sweep: sweep 2 repairs L[2], sweep 3 checks
            assert sweeps == 3
    assert after_first == {0, 1}
