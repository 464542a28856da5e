"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Labels are integers with a unique correct answer (the minimum vertex id of
each component, Section II-A and the Graph Convergence theorem), so every
comparison is bit-exact: tolerance 0, for every operator order, schedule,
write mode, driver, launch geometry and edge order.
"""
import itertools
import os

import numpy as np
import pytest

import graphgen
import oracle
from oracle import contour_model as cm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def contour():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2311_02811_amd as contour
    contour.load()
    return contour


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def solve(contour, src, dst, n, **opts):
    s, d = dev(src), dev(dst)
    labels, st = contour.cc_ex(s, d, n, **opts)
    torch.cuda.synchronize()
    return labels.cpu().numpy(), contour.read_stats(st)


def banner(msg):
    print(msg, flush=True)


MODES = [
    dict(),
    dict(order=1),
    dict(order=3),
    dict(order="full"),
    dict(order=1024),
    dict(order=5),
    dict(write="atomic"),
    dict(order="full", write="atomic"),
    dict(schedule="11mm", order=1024),
    dict(schedule="1m1m", order=1024),
    dict(schedule="11mm", order=2, k1=3),
    dict(driver="hostloop"),
    dict(driver="hostloop", order=1),
    dict(driver="hostloop", order="full", write="atomic"),
    dict(driver="hostloop", update="sync", write="atomic"),
    dict(driver="hostloop", update="sync", write="atomic", order=1),
    dict(driver="hostloop", update="sync", write="atomic", order="full"),
    dict(reorder="on"),
    dict(reorder="on", order="full"),
    dict(reorder="on", driver="hostloop"),
    dict(reorder="on", driver="hostloop", update="sync", write="atomic"),
]
MODE_IDS = ["-".join("%s=%s" % kv for kv in sorted(m.items())) or "default" for m in MODES]

GEOMETRIES = [
    dict(block=256, edges_per_thread=1),
    dict(block=512, edges_per_thread=2),
    dict(block=256, edges_per_thread=8, chunk_tiles=1),
    dict(block=256, edges_per_thread=4, chunk_tiles=3, grid=3),
    dict(block=512, edges_per_thread=4, grid=1),
]


def union_of_all_small_graphs(nmax):
    """Disjoint union of every labelled graph on n <= nmax vertices."""
    src, dst, off = [], [], 0
    for n in range(1, nmax + 1):
        slots = list(itertools.combinations(range(n), 2))
        for mask in range(1 << len(slots)):
            for i, (a, b) in enumerate(slots):
                if mask >> i & 1:
                    src.append(off + b)
                    dst.append(off + a)
            off += n
    return np.array(src, np.int32), np.array(dst, np.int32), off


def test_golden_tiny(contour):
    from tests.test_oracle_pins import TINY
    for name, n, s, d, exp in TINY:
        for mode in MODES:
            banner("tiny %s %r" % (name, mode))
            got, st = solve(contour, s, d, n, **mode)
            assert np.array_equal(got, exp), (name, mode)
            assert st.status == 0


@pytest.mark.parametrize("mode", MODES, ids=MODE_IDS)
def test_every_small_graph(contour, mode):
    src, dst, n = union_of_all_small_graphs(5)
    exp = oracle.uf_labels(src, dst, n)
    banner("all graphs n<=5 as one union (n=%d m=%d) %r" % (n, src.size, mode))
    got, st = solve(contour, src, dst, n, **mode)
    assert np.array_equal(got, exp)
    assert st.status == 0


def test_every_graph_on_six_vertices(contour):
    src, dst, n = union_of_all_small_graphs(6)
    exp = oracle.uf_labels(src, dst, n)
    for mode in (dict(), dict(order=1), dict(order="full"), dict(write="atomic")):
        banner("all graphs n<=6 (n=%d m=%d) %r" % (n, src.size, mode))
        got, _ = solve(contour, src, dst, n, **mode)
        assert np.array_equal(got, exp)


RANDOM_GRAPHS = [
    ("er_sub", lambda: (graphgen.er(65536, 16384, 2), 65536)),
    ("er_crit", lambda: (graphgen.er(65536, 32768, 3), 65536)),
    ("er_super", lambda: (graphgen.er(65536, 65536, 4), 65536)),
    ("grid_rowmajor", lambda: (graphgen.grid_holes(300, 257, 0.1, 5), 300 * 257)),
    ("grid_permuted", lambda: (graphgen.grid_holes(300, 257, 0.1, 6, permute_ids=True), 300 * 257)),
    ("rmat14", lambda: (graphgen.rmat(14, 8, 7), 1 << 14)),
    ("path_up", lambda: ((np.arange(9999, dtype=np.int32), np.arange(1, 10000, dtype=np.int32)), 10000)),
    ("path_down", lambda: ((np.arange(9999, 0, -1, dtype=np.int32),
                            np.arange(9998, -1, -1, dtype=np.int32)), 10000)),
]


@pytest.mark.parametrize("graph", RANDOM_GRAPHS, ids=[g[0] for g in RANDOM_GRAPHS])
def test_random_graphs_all_modes(contour, graph):
    name, make = graph
    (src, dst), n = make()
    exp = oracle.uf_labels(src, dst, n)
    for mode in MODES:
        if name.startswith("path") and mode.get("order") == 1 and mode.get("update") == "sync":
            continue  # 10^4 host-sequenced sweeps: covered by the smaller paths
        banner("%s n=%d m=%d %r" % (name, n, src.size, mode))
        got, st = solve(contour, src, dst, n, **mode)
        assert np.array_equal(got, exp), (name, mode)
        assert st.status == 0 and st.sweeps_executed >= 1


@pytest.mark.parametrize("geom", GEOMETRIES, ids=[str(g) for g in GEOMETRIES])
def test_launch_geometries(contour, geom):
    for name, make in RANDOM_GRAPHS[:6]:
        (src, dst), n = make()
        exp = oracle.uf_labels(src, dst, n)
        for mode in (dict(), dict(order="full"), dict(driver="hostloop")):
            banner("%s %r %r" % (name, geom, mode))
            got, _ = solve(contour, src, dst, n, **geom, **mode)
            assert np.array_equal(got, exp), (name, geom, mode)


def test_ragged_sizes(contour):
    # sizes around tile boundaries (256 threads x 1..8 edges)
    for m in (1, 2, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 2047, 2049, 4097):
        n = max(2, m // 2)
        src, dst = graphgen.er(n, min(m, n * (n - 1) // 2), m)
        exp = oracle.uf_labels(src, dst, n)
        for geom in GEOMETRIES:
            got, _ = solve(contour, src, dst, n, **geom)
            assert np.array_equal(got, exp), (m, geom)


def test_sync_mode_matches_algorithm1_sweep_by_sweep(contour):
    # C-Syn is deterministic: after k iterations the GPU state equals the
    # model of Algorithm 1 after k iterations, for every k.
    for order in (1, 2, 3, cm.FULL):
        src, dst = graphgen.grid_holes(40, 37, 0.15, 9, permute_ids=True)
        n = 40 * 37
        _, iters, _, states = cm.contour_sync(src, dst, n, order, record=True)
        for k in range(1, iters + 1):
            banner("sync order %d after %d of %d iterations" % (order, k, iters))
            got, st = solve(contour, src, dst, n, driver="hostloop", update="sync", write="atomic",
                            order="full" if order == cm.FULL else order, max_sweeps=k)
            assert np.array_equal(got, states[k - 1]), (order, k)
        got, st = solve(contour, src, dst, n, driver="hostloop", update="sync", write="atomic",
                        order="full" if order == cm.FULL else order)
        assert st.sweeps_executed == iters and st.status == 0


@pytest.mark.parametrize("sched,k1", [("11mm", 2), ("1m1m", 2), ("11mm", 3)])
def test_sync_mode_schedules_match_algorithm1_sweep_by_sweep(contour, sched, k1):
    # Operator schedules of Section III-B-4 under the synchronous update: the
    # order changes from one iteration to the next, and after every iteration
    # the GPU state equals the model's (C-11mm with k1 order-1 iterations
    # first, C-1m1m alternating from order 1; the paper's m = 1024).  The path
    # with increasing ids is one of the graphs: its states are the closed
    # forms of tests/golden/schedule_closed_forms.txt.
    graphs = [(np.arange(63, dtype=np.int32), np.arange(1, 64, dtype=np.int32), 64),
              (*graphgen.grid_holes(40, 37, 0.15, 9, permute_ids=True), 40 * 37)]
    name = "C-11mm" if sched == "11mm" else "C-1m1m"
    for src, dst, n in graphs:
        _, iters, _, states = cm.contour_sync(src, dst, n, cm.schedule(name, m=1024, k1=k1), record=True)
        for k in range(1, iters + 1):
            banner("sync %s k1=%d n=%d after %d of %d iterations" % (sched, k1, n, k, iters))
            got, st = solve(contour, src, dst, n, driver="hostloop", update="sync", write="atomic",
                            order=1024, schedule=sched, k1=k1, max_sweeps=k)
            assert np.array_equal(got, states[k - 1]), (sched, k1, n, k)
        got, st = solve(contour, src, dst, n, driver="hostloop", update="sync", write="atomic",
                        order=1024, schedule=sched, k1=k1)
        assert st.sweeps_executed == iters and st.status == 0


def test_edge_cases(contour):
    e = np.zeros(0, np.int32)
    got, st = solve(contour, e, e, 0)
    assert got.size == 0 and st.status == 0
    got, st = solve(contour, e, e, 1)
    assert np.array_equal(got, [0]) and st.sweeps_executed == 0
    got, st = solve(contour, e, e, 7)
    assert np.array_equal(got, np.arange(7))
    got, st = solve(contour, np.array([3, 3, 1], np.int32), np.array([3, 3, 1], np.int32), 5)
    assert np.array_equal(got, np.arange(5)) and st.status == 0
    n = 1 << 20
    got, st = solve(contour, np.array([n - 1], np.int32), np.array([n - 2], np.int32), n)
    exp = np.arange(n, dtype=np.int32)
    exp[n - 1] = n - 2
    assert np.array_equal(got, exp)


@pytest.mark.parametrize("mode", [dict(reorder="on"), dict(reorder="on", write="atomic"),
                                  dict(reorder="on", order="full"), dict(reorder="off")],
                         ids=["window", "window-atomic", "window-full", "flat"])
def test_ids_at_the_top_of_the_window_range(contour, mode):
    # label windows are used up to n = 2^30 - 1 and tag staged labels with
    # bit 30: a graph on ids at the start of the last source block (blocks of
    # 2^20 ids here, so a task's window covers them), everything else
    # isolated
    n = (1 << 30) - 1
    k = 6000
    lo = 1023 << 20
    src, dst = graphgen.er(k, 9000, 41)
    exp = oracle.uf_labels(src, dst, k) + lo
    s, d = dev(src.astype(np.int64) + lo), dev(dst.astype(np.int64) + lo)
    banner("top ids %r" % (mode,))
    labels, st = contour.cc_ex(s, d, n, **mode)
    torch.cuda.synchronize()
    assert contour.read_stats(st).status == 0
    assert np.array_equal(labels[lo:lo + k].cpu().numpy(), exp)
    # everything below is isolated: its own label
    assert bool((labels[:lo] == torch.arange(lo, dtype=torch.int32, device="cuda")).all())
    assert bool((labels[lo + k:] == torch.arange(lo + k, n, dtype=torch.int32, device="cuda")).all())
    del labels
    torch.cuda.empty_cache()


def test_reorder_leaves_inputs_untouched(contour):
    src, dst = graphgen.rmat(16, 8, 3)
    n = 1 << 16
    exp = oracle.uf_labels(src, dst, n)
    s, d = dev(src), dev(dst)
    for mode in (dict(reorder="on"), dict(reorder="on", driver="hostloop"), dict(reorder="off")):
        lab, _ = contour.cc_ex(s, d, n, **mode)
        assert np.array_equal(lab.cpu().numpy(), exp)
        assert np.array_equal(s.cpu().numpy(), src) and np.array_equal(d.cpu().numpy(), dst)


def test_out_of_range_ids_are_skipped_and_reported(contour):
    src = np.array([0, 1, 5, -1, 2], np.int32)
    dst = np.array([1, 2, 0, 3, 3], np.int32)
    for mode in (dict(), dict(driver="hostloop"), dict(order="full"), dict(reorder="on"),
                 dict(reorder="on", driver="hostloop")):
        got, st = solve(contour, src, dst, 5, **mode)
        assert st.status == contour.ERANGE
        # the graph without the bad edges: {0, 1, 2, 3}, {4}
        assert np.array_equal(got, [0, 0, 0, 0, 4])


def test_sweep_limit_and_warm_start_resume(contour):
    src, dst = graphgen.grid_holes(200, 200, 0.1, 12)
    n = 40000
    exp = oracle.uf_labels(src, dst, n)
    for mode in (dict(), dict(driver="hostloop"), dict(order=1)):
        s, d = dev(src), dev(dst)
        lab, st = contour.cc_ex(s, d, n, max_sweeps=1, **mode)
        stats = contour.read_stats(st)
        assert stats.status == contour.ENOCONV and stats.sweeps_executed == 1
        part = lab.cpu().numpy()
        assert not np.array_equal(part, exp)
        # a valid partial state: L[x] <= x and L[x] in x's component
        assert np.all(part <= np.arange(n)) and np.array_equal(exp[part], exp)
        lab2, st2 = contour.cc_ex(s, d, n, labels=lab, warm_start=True, **mode)
        assert np.array_equal(lab2.cpu().numpy(), exp)
        assert contour.read_stats(st2).status == 0


@pytest.mark.parametrize("mode", [dict(), dict(reorder="on"), dict(order=3), dict(order="full"),
                                  dict(write="atomic"), dict(driver="hostloop")],
                         ids=["default", "reorder", "order3", "full", "atomic", "hostloop"])
def test_async_states_keep_the_invariants_sweep_by_sweep(contour, mode):
    # Snapshots of the asynchronous update one sweep at a time (a sweep limit
    # of 1, then a warm start from the snapshot): at every snapshot
    # L[x] <= x and L[x] lies in x's component (the invariants of
    # Section II-A that every conditional assignment keeps), labels never
    # rise from one snapshot to the next, and the chain ends once a sweep
    # leaves the state unchanged, at the oracle's labels.
    for (src, dst), n in ((graphgen.grid_holes(300, 200, 0.1, 4, permute_ids=True), 60000),
                          (graphgen.rmat(16, 8, 6), 1 << 16)):
        exp = oracle.uf_labels(src, dst, n)
        ids = np.arange(n)
        s, d = dev(src), dev(dst)
        lab = torch.arange(n, dtype=torch.int32, device="cuda")
        prev = ids.astype(np.int32)
        for k in range(1, 64):
            banner("snapshot %r n=%d sweep %d" % (mode, n, k))
            lab, st = contour.cc_ex(s, d, n, labels=lab, warm_start=True, max_sweeps=1, **mode)
            torch.cuda.synchronize()
            cur = lab.cpu().numpy()
            stats = contour.read_stats(st)
            assert np.all(cur <= ids) and np.all(cur >= 0), (mode, k)
            assert np.array_equal(exp[cur], exp), (mode, k)
            assert np.all(cur <= prev), (mode, k)
            if stats.status == contour.OK:
                # the sweep found nothing to change: converged
                assert np.array_equal(cur, prev) and np.array_equal(cur, exp), (mode, k)
                break
            assert stats.status == contour.ENOCONV
            prev = cur
        else:
            pytest.fail("no convergence in 63 single-sweep steps")


def test_bad_warm_start_is_rejected(contour):
    src, dst = graphgen.er(100, 200, 1)
    s, d = dev(src), dev(dst)
    bad = torch.arange(100, dtype=torch.int32, device="cuda")
    bad[10] = 50  # L[x] > x
    _, st = contour.cc_ex(s, d, 100, labels=bad, warm_start=True)
    assert contour.read_stats(st).status == contour.EINVAL


def test_invalid_options_are_synchronous_errors(contour):
    src, dst = graphgen.er(100, 200, 1)
    s, d = dev(src), dev(dst)
    with pytest.raises(contour.ContourError) as e:
        contour.cc_ex(s, d, 100, update="sync")          # sync needs atomic + hostloop
    assert e.value.code == contour.ENOTSUP
    with pytest.raises(contour.ContourError) as e:
        contour.cc_ex(s, d, 100, order=0x7fff)
    assert e.value.code == contour.EINVAL
    with pytest.raises(contour.ContourError):
        contour.cc_ex(s, d, -1)


def test_repeatability_under_races(contour):
    # plain stores race by design; 30 runs with shuffled edge orders all reach
    # the same labels
    src, dst = graphgen.grid_holes(512, 512, 0.1, 21)
    n = 512 * 512
    exp = oracle.uf_labels(src, dst, n)
    sweeps = []
    for seed in range(30):
        s2, d2 = src.copy(), dst.copy()
        graphgen.shuffle_edges(s2, d2, seed)
        got, st = solve(contour, s2, d2, n, **(GEOMETRIES[seed % len(GEOMETRIES)]))
        assert np.array_equal(got, exp), seed
        sweeps.append(st.sweeps_executed)
    print("sweeps over 30 runs: min %d max %d" % (min(sweeps), max(sweeps)))


def test_stream_and_concurrency(contour):
    src, dst = graphgen.er(50000, 60000, 5)
    exp = oracle.uf_labels(src, dst, 50000)
    s, d = dev(src), dev(dst)
    streams = [torch.cuda.Stream() for _ in range(3)]
    outs = []
    for st in streams:
        with torch.cuda.stream(st):
            outs.append(contour.cc(s, d, 50000, stream=st))
    torch.cuda.synchronize()
    for o in outs:
        assert np.array_equal(o.cpu().numpy(), exp)


# ------------------------------------------------- destination ranges --
# Edges grouped by destination range and dealt to the XCDs by per-XCD queues
# (CONTOUR_DST_RANGES_*): labels must not depend on it.  Graphs with n above
# 2^20 and m >= 4 n take it by default; smaller range sizes, tiny windows,
# explicit grids (two units per XCD; one workgroup per XCD; more workgroups
# than fit the GPU at once) and a grid that is not a multiple of eight (the
# single-counter fallback) exercise the queues and their stealing.

RANGE_GRAPHS = [
    ("er_n1500000_m8000000", lambda: (graphgen.er(1_500_000, 8_000_000, 21), 1_500_000)),
    ("rmat21_ef16", lambda: (graphgen.rmat(21, 16, 22), 1 << 21)),
    ("grid1100_holes10", lambda: (graphgen.grid_holes(1100, 1100, 0.1, 23), 1100 * 1100)),
]

RANGE_MODES = [
    dict(),
    dict(dst_ranges="on"),
    dict(dst_ranges="off"),
    dict(dst_ranges=16),
    dict(dst_ranges=20, order=3),
    dict(dst_ranges="on", order="full"),
    dict(dst_ranges="on", write="atomic"),
    dict(dst_ranges="on", block=1024, edges_per_thread=2),
    dict(dst_ranges="on", block=1024, edges_per_thread=4),
    dict(dst_ranges="on", window=2048),
    dict(dst_ranges="on", grid=16),
    dict(dst_ranges="on", grid=8),
    dict(dst_ranges="on", grid=1024),
    dict(dst_ranges="on", grid=12),
    dict(dst_ranges="on", schedule="1m1m", order=1024),
]


@pytest.mark.parametrize("graph", RANGE_GRAPHS, ids=[g[0] for g in RANGE_GRAPHS])
def test_destination_ranges(contour, graph):
    name, make = graph
    (src, dst), n = make()
    exp = oracle.uf_labels(src, dst, n)
    s, d = dev(src), dev(dst)
    for mode in RANGE_MODES:
        banner("ranges %s n=%d m=%d %r" % (name, n, src.size, mode))
        lab, st = contour.cc_ex(s, d, n, **mode)
        stats = contour.read_stats(st)
        assert stats.status == contour.OK, mode
        assert np.array_equal(lab.cpu().numpy(), exp), mode
    # one sweep at a time, resumed from each partial state
    lab = torch.arange(n, dtype=torch.int32, device="cuda")
    for k in range(1, 64):
        lab, st = contour.cc_ex(s, d, n, labels=lab, warm_start=True, max_sweeps=1, dst_ranges="on")
        stats = contour.read_stats(st)
        cur = lab.cpu().numpy()
        assert np.all(cur <= np.arange(n)) and np.array_equal(exp[cur], exp), k
        if stats.status == contour.OK:
            break
        assert stats.status == contour.ENOCONV
    assert np.array_equal(lab.cpu().numpy(), exp)


def test_destination_ranges_out_of_range_ids(contour):
    src, dst = graphgen.er(1_200_000, 5_000_000, 24)
    n = 1_200_000
    keep = np.ones(src.size, bool)
    keep[::1001] = False
    exp = oracle.uf_labels(src[keep], dst[keep], n)
    src, dst = src.copy(), dst.copy()
    src[::2002] = -3
    dst[1001::2002] = n + 5
    got, st = solve(contour, src, dst, n, dst_ranges="on")
    assert st.status == contour.ERANGE
    assert np.array_equal(got, exp)


# ------------------------------------------------------------ full size --

def test_config_er_full(contour):
    n, m = 65536, 524288
    src, dst = graphgen.er(n, m, 1)
    exp = oracle.uf_labels(src, dst, n)
    for mode in (dict(), dict(write="atomic"), dict(driver="hostloop"), dict(order=3),
                 dict(order="full")):
        got, st = solve(contour, src, dst, n, **mode)
        assert np.array_equal(got, exp), mode


def test_config_grid_full(contour):
    banner("generating 4096x4096 grid with 10% holes")
    src, dst = graphgen.grid_holes(4096, 4096, 0.1, 1)
    n = 4096 * 4096
    exp = oracle.uf_labels(src, dst, n)
    ncomp = int(np.count_nonzero(exp == np.arange(n)))
    s, d = dev(src), dev(dst)
    for mode in (dict(), dict(order=3), dict(order="full"), dict(write="atomic"),
                 dict(driver="hostloop"), dict(reorder="off"), dict(reorder="on", order=1)):
        banner("grid full %r" % mode)
        lab, st = contour.cc_ex(s, d, n, **mode)
        got = lab.cpu().numpy()
        stats = contour.read_stats(st)
        assert np.array_equal(got, exp), mode
        print("grid %r: %d sweeps (theorem bound for the hole-free lattice: %d), %d components"
              % (mode, stats.sweeps_executed, cm.theorem_bound(8190), ncomp))


def test_config_rmat_full(contour):
    banner("generating R-MAT scale 24, edge factor 16")
    src, dst = graphgen.rmat(24, 16, 1)
    n = 1 << 24
    exp = oracle.uf_labels(src, dst, n)
    s, d = dev(src), dev(dst)
    del src, dst
    for mode in (dict(), dict(order=3), dict(order="full"), dict(reorder="off"), dict(dst_ranges="off"),
                 dict(dst_ranges=20), dict(driver="hostloop"), dict(driver="hostloop", order=3)):
        banner("rmat full %r" % mode)
        lab, st = contour.cc_ex(s, d, n, **mode)
        assert np.array_equal(lab.cpu().numpy(), exp), mode
        print("rmat %r: %d sweeps" % (mode, contour.read_stats(st).sweeps_executed))


def test_count_reads_at_the_fixed_point(contour):
    # contour_cc_count_reads counts the chain reads of orders above 3 and
    # chase-to-root.  Warm-started from the exact labels, the solve is one
    # sweep that changes nothing, so the count is fixed: a chain from x reads
    # L[x] and, when x is not a root, L[L[x]] = L[x] as well -- one read from
    # a root, two from any other vertex, for both endpoints of every edge.
    for (src, dst), n in ((graphgen.grid_holes(300, 200, 0.1, 31), 60000),
                          (graphgen.rmat(16, 8, 32), 1 << 16),
                          (graphgen.rmat(21, 16, 33), 1 << 21)):
        exp = oracle.uf_labels(src, dst, n)
        root = exp == np.arange(n)
        want = int(np.sum(np.where(root[src], 1, 2)) + np.sum(np.where(root[dst], 1, 2)))
        s, d = dev(src), dev(dst)
        for mode in (dict(order="full"), dict(order=5), dict(order="full", reorder="on"),
                     dict(order="full", dst_ranges="on")):
            lab = dev(exp)
            lab, st, reads = contour.cc_count_reads(s, d, n, labels=lab, warm_start=True, **mode)
            stats = contour.read_stats(st)
            banner("count reads n=%d m=%d %r: %d" % (n, src.size, mode, int(reads.item())))
            assert stats.status == 0 and stats.sweeps_executed == 1 and stats.sweeps_with_writes == 0
            assert np.array_equal(lab.cpu().numpy(), exp)
            assert int(reads.item()) == want, mode
        # orders up to 3 are not counted; a cold solve counts at least one read per endpoint and sweep
        _, _, reads = contour.cc_count_reads(s, d, n, order=2)
        assert int(reads.item()) == 0
        _, st, reads = contour.cc_count_reads(s, d, n, order="full")
        assert int(reads.item()) >= 2 * src.size * contour.read_stats(st).sweeps_executed


def test_gather_ceiling_measurement_kernel(contour):
    # contour_gather_ceiling only reads: every mode returns OK and leaves the
    # labels and edges as they were (aligned and unaligned edge arrays, a
    # ragged tail, ids outside [0, n))
    import ctypes
    lib = contour.load()
    src, dst = graphgen.rmat(16, 8, 41)
    src[::101] = -1
    n = 1 << 16
    s, d = dev(src), dev(dst)
    labels = torch.arange(n, dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for off in (0, 1):
        m = src.size - 3 - off
        for mode in (0, 1, 2):
            rc = lib.contour_gather_ceiling(ctypes.c_void_p(s.data_ptr() + 4 * off), ctypes.c_void_p(d.data_ptr() + 4 * off),
                                            m, ctypes.c_void_p(labels.data_ptr()), n, mode,
                                            ctypes.c_void_p(sink.data_ptr()), stream)
            assert rc == contour.OK
    torch.cuda.synchronize()
    assert torch.equal(labels.cpu(), torch.arange(n, dtype=torch.int32))
    assert np.array_equal(s.cpu().numpy(), src) and np.array_equal(d.cpu().numpy(), dst)
