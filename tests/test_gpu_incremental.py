"""GPU tests of contour_cc_add_edges and the Graph front end.

Edges arrive in batches; after every batch the labels must equal the
oracle's labels of all edges so far, bit for bit (tolerance 0: labels are
integers with a unique correct answer).  The CPU model of the same scheme
(oracle/contour_model.add_edges) is pinned in tests/test_contour_model.py.
"""
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


def graph(kind, seed):
    if kind == "er":
        s, d = graphgen.er(5000, 6000, seed)
        return s, d, 5000
    if kind == "grid":
        s, d = graphgen.grid_holes(100, 120, 0.3, seed)
        return s, d, 100 * 120
    s, d = graphgen.rmat(14, 4, seed)
    return s, d, 1 << 14


MODES = [dict(), dict(order=1), dict(order=3), dict(order="full"), dict(write="atomic"),
         dict(driver="hostloop"), dict(reorder="on"), dict(update="sync", driver="hostloop", write="atomic")]


@pytest.mark.parametrize("mode", MODES, ids=[str(m) for m in MODES])
@pytest.mark.parametrize("kind", ["er", "grid", "rmat"])
def test_batches_of_edges_match_oracle(contour, kind, mode):
    src, dst, n = graph(kind, 31)
    rng = np.random.default_rng(7)
    cuts = np.sort(rng.integers(0, src.size + 1, 6))
    bounds = [0, *cuts.tolist(), src.size]
    print("incremental", kind, mode, "batches", len(bounds) - 1, flush=True)
    L = torch.arange(n, dtype=torch.int32, device="cuda")
    for a, b in zip(bounds[:-1], bounds[1:]):
        _, st = contour.add_edges(dev(src[a:b]), dev(dst[a:b]), n, L, **mode)
        assert contour.read_stats(st).status == 0
        assert np.array_equal(L.cpu().numpy(), oracle.uf_labels(src[:b], dst[:b], n)), (a, b)


def test_graph_front_end(contour):
    src, dst, n = graph("grid", 5)
    g = contour.Graph(n)
    assert g.num_components() == n
    step = 997
    for a in range(0, src.size, step):
        g.add_edges(dev(src[a:a + step]), dev(dst[a:a + step]))
    exp = oracle.uf_labels(src, dst, n)
    assert np.array_equal(g.labels.cpu().numpy(), exp)
    assert g.num_components() == len(np.unique(exp))
    assert g.num_edges == src.size
    u, v = int(src[0]), int(dst[0])
    assert g.connected(u, v)


def test_add_edges_edge_cases(contour):
    n = 10
    L = torch.arange(n, dtype=torch.int32, device="cuda")
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    _, st = contour.add_edges(e, e, n, L)                  # no new edges: nothing changes
    assert contour.read_stats(st).status == 0
    assert torch.equal(L.cpu(), torch.arange(n, dtype=torch.int32))
    _, st = contour.add_edges(dev([3, 7]), dev([9, 12]), n, L)   # one id out of range
    assert contour.read_stats(st).status == contour.ERANGE
    assert np.array_equal(L.cpu().numpy(), oracle.uf_labels(np.array([3]), np.array([9]), n))
    bad = torch.tensor([0, 5, 2, 3, 4, 5, 6, 7, 8, 9], dtype=torch.int32, device="cuda")  # L[1] > 1
    before = bad.clone()
    _, st = contour.add_edges(dev([1]), dev([2]), n, bad)
    assert contour.read_stats(st).status == contour.EINVAL
    assert torch.equal(bad, before)


def test_add_edges_large_grid_matches_full_solve(contour):
    # the headline grid in two halves against one solve of all edges
    src, dst = graphgen.grid_holes(2048, 2048, 0.1, 3)
    n = 2048 * 2048
    h = src.size // 2
    L = contour.cc(dev(src[:h]), dev(dst[:h]), n)
    _, st = contour.add_edges(dev(src[h:]), dev(dst[h:]), n, L)
    assert contour.read_stats(st).status == 0
    full = contour.cc(dev(src), dev(dst), n)
    assert torch.equal(L, full)
    assert np.array_equal(L.cpu().numpy(), oracle.uf_labels(src, dst, n))
