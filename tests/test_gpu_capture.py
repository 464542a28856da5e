"""A single-graph solve captured into a hipGraph after contour_reserve.

contour_reserve sizes the stream's workspace up front, so contour_cc_ex then
enqueues only kernels (no allocation, no synchronisation, no memset) and can
be captured.  Each replay must give the oracle's labels bit for bit, with
eager work and synchronisations between the replays.
"""
import ctypes

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


CASES = [
    # grouped edges with label windows (n > 2^20)
    ("grid1100_holes10", lambda: (graphgen.grid_holes(1100, 1100, 0.1, 7), 1100 * 1100), dict()),
    # small graph, not grouped, chase-to-root
    ("er_n20000_m30000", lambda: (graphgen.er(20000, 30000, 8), 20000), dict(order="full")),
]


@pytest.mark.parametrize("name,make,opts", CASES, ids=[c[0] for c in CASES])
def test_captured_solve_replays_exactly(contour, name, make, opts):
    (src, dst), n = make()
    print("capture case", name, "m=%d" % src.size, opts, flush=True)
    expect = oracle.uf_labels(src, dst, n)
    s, d = dev(src), dev(dst)
    lib = contour.load()
    stream = torch.cuda.Stream()
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    stats = torch.zeros(4, dtype=torch.int32, device="cuda")
    o = contour.make_opts(**opts)
    contour.reserve(src.size, n, stream=stream, **opts)

    def call():
        return lib.contour_cc_ex(ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(d.data_ptr()), src.size, n,
                                 ctypes.c_void_p(labels.data_ptr()), ctypes.byref(o),
                                 ctypes.c_void_p(stats.data_ptr()), ctypes.c_void_p(stream.cuda_stream))

    # one eager solve on the stream first
    with torch.cuda.stream(stream):
        assert call() == contour.OK
    torch.cuda.synchronize()
    assert np.array_equal(labels.cpu().numpy(), expect)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        assert call() == contour.OK
    for rep in range(3):
        labels.fill_(-1)
        stats.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        st = contour.read_stats(stats)
        assert st.status == contour.OK, rep
        assert st.sweeps_executed >= 1
        assert np.array_equal(labels.cpu().numpy(), expect), rep

