"""GPU test of the multi-GPU design's combine rule, run on one GPU.

The design splits the edge list over p GPUs, each holding the whole label
array; every round each GPU solves its share starting from the current
labels (a warm-started contour_cc_ex) and the p label arrays are combined by
an elementwise minimum.  Here the p shares are solved one after the other on
the same GPU and merged with contour_merge_min (checked against torch's
elementwise minimum and its count of lowered labels): the final labels must equal
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
        Ln = outs[0].clone()
        lowered = 0
        for Li in outs[1:]:
            expect = int((Li < Ln).sum())
            cnt = contour.merge_min(Li, Ln)
            assert int(cnt.item()) == expect
            lowered += expect
        assert torch.equal(Ln, torch.stack(outs).min(dim=0).values)
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


@pytest.mark.parametrize("n", [1, 3, 4, 5, 1000, (1 << 20) + 3])
@pytest.mark.parametrize("offset", [0, 1])
def test_merge_min_matches_elementwise_minimum(contour, n, offset):
    # aligned arrays take four labels per load, offset ones the scalar path;
    # both cover a ragged tail
    g = torch.Generator().manual_seed(n * 2 + offset)
    a = torch.randint(0, max(n, 2), (n + offset,), generator=g, dtype=torch.int32).cuda()
    b = torch.randint(0, max(n, 2), (n + offset,), generator=g, dtype=torch.int32).cuda()
    peer, lab = a[offset:], b[offset:]
    want = torch.minimum(peer, lab)
    expect = int((peer < lab).sum())
    before = b[:offset].clone()
    print("merge_min n", n, "offset", offset, flush=True)
    cnt = contour.merge_min(peer, lab)
    torch.cuda.synchronize()
    assert torch.equal(lab, want)
    assert int(cnt.item()) == expect
    assert torch.equal(b[:offset], before)  # nothing before the view is touched
    # a second merge of the same peer changes nothing; merging with itself neither
    assert int(contour.merge_min(peer, lab).item()) == 0
    assert int(contour.merge_min(lab, lab).item()) == 0
    assert torch.equal(lab, want)


def test_merge_min_of_two_label_states_at_full_size(contour):
    # two valid states of the R-MAT scale-24 label array (labels at or below
    # their ids): the merge is their elementwise minimum, and merging the
    # result into either one again lowers nothing
    n = 1 << 24
    idx = torch.arange(n, dtype=torch.int32, device="cuda")
    g = torch.Generator(device="cuda").manual_seed(3)
    la = (idx - torch.randint(0, 64, (n,), device="cuda", generator=g, dtype=torch.int32)).clamp_min(0)
    lb = (idx - torch.randint(0, 64, (n,), device="cuda", generator=g, dtype=torch.int32)).clamp_min(0)
    want = torch.minimum(la, lb)
    expect = int((lb < la).sum())
    print("merge_min full size", n, flush=True)
    cnt = contour.merge_min(lb, la)
    assert torch.equal(la, want)
    assert int(cnt.item()) == expect
    assert bool((la <= idx).all())
    assert int(contour.merge_min(lb, la).item()) == 0
    assert contour.merge_min(lb, la, count=False) is None
