"""GPU test of the multi-GPU design's combine rule, run on one GPU.

The design splits the edge list over p GPUs, each holding the whole label
array; every round each GPU solves its share starting from the current
labels (a warm-started contour_cc_ex) and the p label arrays are combined by
an elementwise minimum.  Here the p shares are solved one after the other on
the same GPU and the minimum is taken with torch: the final labels must equal
the oracle's for the whole graph (tolerance 0), and the round count must
match the CPU model (oracle/contour_model.sharded_rounds) run on the same
shares, up to the asynchronous sweeps converging differently inside a round
(so only the labels are compared exactly).
"""
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


def rounds_on_one_gpu(contour, src, dst, n, share, p, **opts):
    s = torch.from_numpy(np.ascontiguousarray(src, np.int32)).cuda()
    d = torch.from_numpy(np.ascontiguousarray(dst, np.int32)).cuda()
    sh = torch.from_numpy(np.asarray(share, np.int64)).cuda()
    parts = [(s[sh == i].contiguous(), d[sh == i].contiguous()) for i in range(p)]
    L = torch.arange(n, dtype=torch.int32, device="cuda")
    for r in range(1, 257):
        outs = []
        for ps, pd in parts:
            Li = L.clone()
            _, st = contour.cc_ex(ps, pd, n, labels=Li, warm_start=True, **opts)
            assert contour.read_stats(st).status == 0
            outs.append(Li)
        Ln = torch.stack(outs).min(dim=0).values
        # every round keeps L[x] <= x and never raises a label
        assert bool((Ln <= torch.arange(n, dtype=torch.int32, device="cuda")).all())
        assert bool((Ln <= L).all())
        if torch.equal(Ln, L):
            return L.cpu().numpy(), r
        L = Ln
    raise AssertionError("no convergence in 256 rounds")


@pytest.mark.parametrize("p", [2, 8])
@pytest.mark.parametrize("kind", ["rmat", "grid"])
def test_sharded_rounds_match_oracle(contour, kind, p):
    if kind == "rmat":
        src, dst = graphgen.rmat(16, 8, 21)
        n = 1 << 16
    else:
        src, dst = graphgen.grid_holes(256, 256, 0.1, 22)
        n = 256 * 256
    share = np.random.default_rng(100 + p).integers(0, p, src.size)
    print("sharded", kind, "p", p, "m", src.size, flush=True)
    labels, rounds = rounds_on_one_gpu(contour, src, dst, n, share, p)
    assert np.array_equal(labels, oracle.uf_labels(src, dst, n))
    assert rounds >= 2


def test_sharded_rounds_small_graph_against_model(contour):
    # a graph small enough for the CPU model: same shares, same final labels
    src, dst = graphgen.grid_holes(20, 30, 0.25, 7)
    n = 600
    share = np.random.default_rng(5).integers(0, 3, src.size)
    labels, rounds = rounds_on_one_gpu(contour, src, dst, n, share, 3)
    model, model_rounds, _ = cm.sharded_rounds(src, dst, n, share, 3)
    assert np.array_equal(labels, model)
    assert np.array_equal(labels, oracle.uf_labels(src, dst, n))
