"""GPU parity of the batched path: every graph of a CSR-of-graphs batch gets
exactly its own minimum-id labels (local ids), identical to the CPU oracle and
to a standalone solve of that graph, whatever the batch around it."""
import numpy as np
import pytest

import graphgen
import oracle

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


def banner(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def small_batch():
    # sizes spread so that all three classes appear with the tuning below
    b = graphgen.batch(400, 5, median=400, sigma=1.6, n_lo=1, n_hi=300000)
    exp = oracle.uf_batch(b.edge_off, b.vertex_off, b.src, b.dst)
    return b, exp


FORCE_CLASSES = dict(lds_max_vertices=1500, wg_max_edges=30000)


def graphgen_batch(eo, vo, src, dst):
    """The CSR-of-graphs fields run_plan reads, for a hand-made batch."""
    import types
    return types.SimpleNamespace(edge_off=np.asarray(eo, np.int64), vertex_off=np.asarray(vo, np.int64),
                                 src=np.ascontiguousarray(src, np.int32), dst=np.ascontiguousarray(dst, np.int32))


def run_plan(contour, b, tuning=None, **opts):
    s, d = dev(b.src), dev(b.dst)
    plan = contour.BatchPlan(b.edge_off, b.vertex_off, s, d, tuning=tuning, **opts)
    plan.launch()
    torch.cuda.synchronize()
    out = plan.labels.cpu().numpy(), plan.stats.cpu().numpy(), plan.classes()
    plan.close()
    return out


@pytest.mark.parametrize("opts", [dict(), dict(order=1), dict(order=3), dict(order="full"),
                                  dict(write="atomic"), dict(schedule="1m1m", order=1024)],
                         ids=["default", "order1", "order3", "full", "atomic", "1m1m"])
def test_batch_matches_oracle_all_classes(contour, small_batch, opts):
    b, exp = small_batch
    tuning = contour.make_tuning(**FORCE_CLASSES)
    banner("batch G=%d classes forced %r" % (b.num_graphs, opts))
    labels, stats, classes = run_plan(contour, b, tuning=tuning, **opts)
    assert all(c > 0 for c in classes), classes
    assert np.array_equal(labels, exp)
    assert np.all(stats[:, 0] == 0)
    assert np.all(stats[b.m > 0, 1] >= 1)


def test_batch_tuned_geometries(contour, small_batch):
    b, exp = small_batch
    for spec in ([dict(block=256, edges_per_thread=1), dict(block=1024, edges_per_thread=4),
                  dict(block=512, edges_per_thread=8)],
                 [dict(block=1024, edges_per_thread=2, order=3), dict(block=256, edges_per_thread=1,
                                                                      order="full"),
                  dict(block=256, edges_per_thread=1, order=2)]):
        tuning = contour.make_tuning(spec, **FORCE_CLASSES)
        banner("batch tuned %r" % spec)
        labels, stats, _ = run_plan(contour, b, tuning=tuning)
        assert np.array_equal(labels, exp)


def test_batch_slice_equals_standalone(contour, small_batch):
    b, exp = small_batch
    labels, _, _ = run_plan(contour, b, tuning=contour.make_tuning(**FORCE_CLASSES))
    for g in range(0, b.num_graphs, 37):
        s, d, n = b.graph(g)
        v0 = int(b.vertex_off[g])
        alone = contour.cc(dev(s), dev(d), n).cpu().numpy() if n else np.empty(0, np.int32)
        assert np.array_equal(labels[v0:v0 + n], alone), g


def test_batch_edge_cases(contour):
    # empty graphs, edgeless graphs, a single vertex, duplicates and self-loops
    graphs = [(0, []), (1, []), (3, []), (2, [(1, 0), (0, 1), (1, 1)]), (5, [(4, 3), (3, 2)]),
              (70000, [(69999, 0)])]
    src, dst, eo, vo = [], [], [0], [0]
    for n, edges in graphs:
        for a, c in edges:
            src.append(a)
            dst.append(c)
        eo.append(len(src))
        vo.append(vo[-1] + n)
    src = np.array(src, np.int32)
    dst = np.array(dst, np.int32)
    exp = oracle.uf_batch(eo, vo, src, dst)
    plan = contour.BatchPlan(eo, vo, dev(src), dev(dst))
    plan.launch()
    torch.cuda.synchronize()
    assert np.array_equal(plan.labels.cpu().numpy(), exp)
    st = plan.stats.cpu().numpy()
    assert np.all(st[:, 0] == 0)
    assert st[0, 1] == 0 and st[1, 1] == 0
    plan.close()
    # a batch with no graphs at all
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    plan = contour.BatchPlan([0], [0], e, e)
    plan.launch()
    torch.cuda.synchronize()
    plan.close()


def test_batch_out_of_range_local_id(contour):
    src = np.array([0, 5, 1], np.int32)     # graph 1 has n = 3: id 5 is out of range
    dst = np.array([1, 0, 2], np.int32)
    eo, vo = [0, 1, 3], [0, 2, 5]
    plan = contour.BatchPlan(eo, vo, dev(src), dev(dst))
    plan.launch()
    torch.cuda.synchronize()
    st = plan.stats.cpu().numpy()
    assert st[0, 0] == 0 and st[1, 0] == contour.ERANGE
    assert np.array_equal(plan.labels.cpu().numpy(), [0, 0, 0, 1, 1])
    plan.close()


def test_plan_relaunch_and_graph_capture(contour, small_batch):
    b, exp = small_batch
    s, d = dev(b.src), dev(b.dst)
    plan = contour.BatchPlan(b.edge_off, b.vertex_off, s, d,
                             tuning=contour.make_tuning(**FORCE_CLASSES))
    for _ in range(3):
        plan.labels.fill_(-1)
        plan.launch()
        torch.cuda.synchronize()
        assert np.array_equal(plan.labels.cpu().numpy(), exp)
    # capture one launch into a graph and replay it, with eager work between
    side = torch.cuda.Stream()
    plan.launch(side)            # warm-up on a non-default stream before capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch()
    for rep in range(4):
        plan.labels.fill_(-1)
        x = torch.arange(1000, device="cuda").sum()   # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert int(x) == 499500
        banner("graph replay %d" % rep)
        assert np.array_equal(plan.labels.cpu().numpy(), exp), rep
    plan.close()


def test_batched_config_full(contour):
    banner("generating the 20,000-graph batch")
    b = graphgen.batch(20000, 1)
    exp = oracle.uf_batch(b.edge_off, b.vertex_off, b.src, b.dst)
    s, d = dev(b.src), dev(b.dst)
    plan = contour.BatchPlan(b.edge_off, b.vertex_off, s, d)
    banner("classes %r" % plan.classes())
    plan.launch()
    torch.cuda.synchronize()
    assert np.array_equal(plan.labels.cpu().numpy(), exp)
    st = plan.stats.cpu().numpy()
    assert np.all(st[:, 0] == 0)
    print("batch sweeps: max %d mean %.2f" % (st[:, 1].max(), st[:, 1].mean()))
    plan.close()


@pytest.mark.parametrize("spec", [
    [dict(order=2), dict(order=2), dict(order="full", block=512, edges_per_thread=4)],
    [dict(order=2), dict(order=2), dict(order=2, block=512, edges_per_thread=4)],
    [dict(order=2), dict(order=2), dict(order=2, block=256, edges_per_thread=8)],
], ids=["full-512x4", "2-512x4", "2-256x8"])
def test_batched_many_multi_workgroup_graphs_repeated(contour, spec):
    # ~900 graphs solved by several workgroups each (class 2), with
    # workgroups moving between graphs, checked on every one of several
    # launches.  A regression test of a race on the persistent loop's task
    # word when a task has no barrier inside (no label window): a slow wave
    # could read the next task instead of the current one, skip edges, and
    # let a sweep pass as unchanged too early.
    banner("generating the 20,000-graph batch")
    b = graphgen.batch(20000, 1)
    exp = oracle.uf_batch(b.edge_off, b.vertex_off, b.src, b.dst)
    s, d = dev(b.src), dev(b.dst)
    plan = contour.BatchPlan(b.edge_off, b.vertex_off, s, d,
                             tuning=contour.make_tuning(spec, 16384, 65536))
    banner("classes %r" % plan.classes())
    assert plan.classes()[2] > 500
    for rep in range(4):
        plan.launch()
        torch.cuda.synchronize()
        assert np.array_equal(plan.labels.cpu().numpy(), exp), rep
    plan.close()


def test_single_graph_persistent_without_window_repeated(contour):
    # the same loop on one graph, no reordering (tasks without barriers)
    src, dst = graphgen.er(200000, 1600000, 17)
    s, d = dev(src), dev(dst)
    exp = oracle.uf_labels(src, dst, 200000)
    for geo in (dict(block=512, edges_per_thread=4), dict(block=1024, edges_per_thread=4),
                dict(block=256, edges_per_thread=8)):
        for rep in range(10):
            labels, st = contour.cc_ex(s, d, 200000, reorder="off", **geo)
            assert np.array_equal(labels.cpu().numpy(), exp), (geo, rep)


def test_class0_split_by_lds_size_with_graph_capture(contour):
    # default bounds: class 0 holds graphs up to the whole LDS of a workgroup
    # and runs graphs above 16384 vertices in a launch of their own; class 1
    # runs beside them on the caller's stream
    parts = [graphgen.grid_holes(150, 150, 0.1, 31), graphgen.er(30000, 60000, 32),
             graphgen.grid_holes(130, 300, 0.05, 33), graphgen.er(90000, 200000, 34)]
    ns = [22500, 30000, 39000, 90000]
    for i in range(300):
        parts.append(graphgen.er(50 + 7 * i, 3 * (50 + 7 * i), 100 + i))
        ns.append(50 + 7 * i)
    eo, vo = [0], [0]
    for (s_, d_), n in zip(parts, ns):
        eo.append(eo[-1] + s_.size)
        vo.append(vo[-1] + n)
    src = np.concatenate([p[0] for p in parts]).astype(np.int32)
    dst = np.concatenate([p[1] for p in parts]).astype(np.int32)
    exp = oracle.uf_batch(eo, vo, src, dst)
    plan = contour.BatchPlan(eo, vo, dev(src), dev(dst))
    banner("classes %r" % plan.classes())
    assert plan.classes() == [303, 1, 0]
    plan.launch()
    torch.cuda.synchronize()
    assert np.array_equal(plan.labels.cpu().numpy(), exp)
    assert np.all(plan.stats.cpu().numpy()[:, 0] == 0)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch()
    for rep in range(3):
        plan.labels.fill_(-1)
        x = torch.arange(1000, device="cuda").sum()   # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert int(x) == 499500
        assert np.array_equal(plan.labels.cpu().numpy(), exp), rep
    plan.close()


@pytest.mark.parametrize("opts", [dict(), dict(order=1), dict(order=3), dict(order="full"),
                                  dict(write="atomic")],
                         ids=["default", "order1", "order3", "full", "atomic"])
def test_class1_window_and_global_labels(contour, opts):
    # every graph in class 1 (one workgroup, the lowest ~40 K ids in LDS, the
    # rest in global memory): graphs well above the window, one exactly at its
    # edge, ids permuted so that components' minima fall on both sides
    parts, ns = [], []
    for i, (kind, n) in enumerate([("er", 120000), ("grid", 300 * 400), ("er", 40704), ("er", 40705),
                                   ("grid", 90 * 1000), ("er", 250000), ("er", 3000)]):
        if kind == "er":
            s_, d_ = graphgen.er(n, int(1.2 * n), 40 + i)
        else:
            r = 300 if n == 120000 else 90
            s_, d_ = graphgen.grid_holes(r, n // r, 0.15, 40 + i, permute_ids=True)
        parts.append((s_, d_))
        ns.append(n)
    eo, vo = [0], [0]
    for (s_, d_), n in zip(parts, ns):
        eo.append(eo[-1] + s_.size)
        vo.append(vo[-1] + n)
    src = np.concatenate([p[0] for p in parts]).astype(np.int32)
    dst = np.concatenate([p[1] for p in parts]).astype(np.int32)
    exp = oracle.uf_batch(eo, vo, src, dst)
    banner("class-1 window batch %r" % opts)
    labels, stats, classes = run_plan(contour, graphgen_batch(eo, vo, src, dst),
                                      tuning=contour.make_tuning(None, 64, 1 << 22), **opts)
    assert classes == [0, 7, 0]
    assert np.array_equal(labels, exp)
    assert np.all(stats[:, 0] == 0)


def test_class1_window_out_of_range_ids(contour):
    # a class-1 graph with bad ids below and above the window: they are
    # skipped and reported, the other edges solved
    n = 60000
    s_, d_ = graphgen.er(n, 100000, 50)
    s_ = s_.copy()
    d_ = d_.copy()
    s_[7] = n + 3
    d_[11] = -1
    d_[13] = 1 << 30
    keep = np.ones(s_.size, bool)
    keep[[7, 11, 13]] = False
    exp = oracle.uf_labels(s_[keep], d_[keep], n)
    labels, stats, classes = run_plan(contour, graphgen_batch([0, s_.size], [0, n], s_, d_),
                                      tuning=contour.make_tuning(None, 64, 1 << 22))
    assert classes == [0, 1, 0]
    assert stats[0, 0] == contour.ERANGE
    assert np.array_equal(labels, exp)


def test_explicit_options_override_the_tuning(contour):
    # Non-zero opts fields take precedence over the tuning table.  Paths with
    # increasing ids: order 1 needs many more sweeps than order 2, so the
    # sweep counts show which order the plan ran.
    n, G = 3000, 3
    src = np.concatenate([np.arange(n - 1, dtype=np.int32)] * G)
    dst = src + 1
    eo = np.arange(G + 1, dtype=np.int64) * (n - 1)
    vo = np.arange(G + 1, dtype=np.int64) * n
    exp = oracle.uf_batch(eo, vo, src, dst)
    s, d = dev(src), dev(dst)
    tuning = contour.make_tuning([dict(order=2)] * 3)
    sweeps = {}
    for key, opts in (("tuned", dict()), ("explicit", dict(order=1)), ("explicit_block", dict(order=1, block=256))):
        banner("plan with tuning order 2, opts %r" % opts)
        plan = contour.BatchPlan(eo, vo, s, d, tuning=tuning, **opts)
        plan.launch()
        torch.cuda.synchronize()
        assert np.array_equal(plan.labels.cpu().numpy(), exp), key
        sweeps[key] = int(plan.stats[:, 1].max().item())
        plan.close()
    print("sweeps", sweeps)
    assert sweeps["explicit"] > 3 * sweeps["tuned"]
    assert sweeps["explicit_block"] > 3 * sweeps["tuned"]
