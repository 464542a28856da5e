"""contour_cc_noalloc, the entry point that allocates nothing, through the C ABI.

Its labels must equal those of contour_cc_ex (and the oracle's) bit for bit,
on two calls in a row that share the fixed scratch array, the second with a
smaller input; grouping that does not fit the array is refused with
CONTOUR_REORDER_ON and skipped with CONTOUR_REORDER_AUTO.
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


def call_noalloc(contour, s, d, n, labels, stats, stream, **opts):
    o = contour.make_opts(**opts)
    return contour.load().contour_cc_noalloc(
        ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(d.data_ptr()), s.numel(), n,
        ctypes.c_void_p(labels.data_ptr()), ctypes.byref(o),
        ctypes.c_void_p(stats.data_ptr() if stats is not None else 0), ctypes.c_void_p(stream.cuda_stream))


def reference(contour, s, d, n, **opts):
    labels, st = contour.cc_ex(s, d, n, **opts)
    torch.cuda.synchronize()
    return labels.cpu().numpy(), contour.read_stats(st)


def grouped_bytes(m):
    # grouped copy (2 x m ints, each array padded to 4) plus the count tables
    chunks = (m + 8191) // 8192
    return 4 * (2 * ((m + 3) & ~3) + (chunks + (chunks + 127) // 128) * 1024)


SCRATCH = 32 << 20


def test_two_calls_in_a_row_match_contour_cc_ex(contour):
    stream = torch.cuda.Stream()
    cases = [
        # first: a grid large enough to be grouped, its copy close to the limit
        ("grid1300_holes10", graphgen.grid_holes(1300, 1300, 0.1, 3), 1300 * 1300, dict()),
        # second: smaller, also grouped, another order
        ("er_n1200000_m1100000", graphgen.er(1_200_000, 1_100_000, 4), 1_200_000, dict(order=3)),
    ]
    for name, (src, dst), n, opts in cases:
        print("noalloc case", name, "m=%d" % src.size, opts, flush=True)
        assert grouped_bytes(src.size) + 256 <= SCRATCH
        s, d = dev(src), dev(dst)
        want, want_st = reference(contour, s, d, n, **opts)
        labels = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        stats = torch.zeros(4, dtype=torch.int32, device="cuda")
        with torch.cuda.stream(stream):
            rc = call_noalloc(contour, s, d, n, labels, stats, stream, **opts)
        assert rc == contour.OK
        stream.synchronize()
        got = labels.cpu().numpy()
        st = contour.read_stats(stats)
        assert st.status == want_st.status == contour.OK
        assert st.sweeps_executed >= 1
        assert np.array_equal(got, want)
        assert np.array_equal(got, oracle.uf_labels(src, dst, n))


def test_no_device_memory_is_allocated(contour):
    stream = torch.cuda.Stream()
    src, dst = graphgen.er(1_100_000, 1_200_000, 5)
    n = 1_100_000
    s, d = dev(src), dev(dst)
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    stats = torch.zeros(4, dtype=torch.int32, device="cuda")
    small_s, small_d = dev(src[:4000] % 3000), dev(dst[:4000] % 3000)
    small_l = torch.empty(3000, dtype=torch.int32, device="cuda")
    # warm-up: loads the code objects (and with them the fixed array)
    with torch.cuda.stream(stream):
        assert call_noalloc(contour, s, d, n, labels, stats, stream) == contour.OK
        assert call_noalloc(contour, small_s, small_d, 3000, small_l, stats, stream) == contour.OK
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    with torch.cuda.stream(stream):
        for _ in range(3):
            assert call_noalloc(contour, s, d, n, labels, stats, stream) == contour.OK
            assert call_noalloc(contour, small_s, small_d, 3000, small_l, None, stream) == contour.OK
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free0 - free1 < (1 << 20)
    assert np.array_equal(labels.cpu().numpy(), oracle.uf_labels(src, dst, n))
    assert np.array_equal(small_l.cpu().numpy(), oracle.uf_labels(src[:4000] % 3000, dst[:4000] % 3000, 3000))


def test_grouping_beyond_the_scratch(contour):
    stream = torch.cuda.Stream()
    n = 1_500_000
    src, dst = graphgen.er(n, 4_200_000, 6)
    assert grouped_bytes(src.size) + 256 > SCRATCH
    s, d = dev(src), dev(dst)
    labels = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    stats = torch.zeros(4, dtype=torch.int32, device="cuda")
    print("noalloc beyond the scratch m=%d" % src.size, flush=True)
    # refused synchronously when grouping is required: nothing enqueued
    with torch.cuda.stream(stream):
        assert call_noalloc(contour, s, d, n, labels, stats, stream, reorder="on") == contour.ETOOBIG
    stream.synchronize()
    assert int(labels[0].item()) == -7
    # solved without grouping when it is automatic
    with torch.cuda.stream(stream):
        assert call_noalloc(contour, s, d, n, labels, stats, stream) == contour.OK
    stream.synchronize()
    assert contour.read_stats(stats).status == contour.OK
    assert np.array_equal(labels.cpu().numpy(), oracle.uf_labels(src, dst, n))


def test_degenerate_inputs_and_options(contour):
    stream = torch.cuda.Stream()
    lib = contour.load()
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    labels = torch.full((5,), -1, dtype=torch.int32, device="cuda")
    stats = torch.full((4,), -1, dtype=torch.int32, device="cuda")
    with torch.cuda.stream(stream):
        # m = 0: identity labels, no sweep
        assert call_noalloc(contour, e, e, 5, labels, stats, stream) == contour.OK
    stream.synchronize()
    assert labels.tolist() == [0, 1, 2, 3, 4]
    assert contour.read_stats(stats).status == contour.OK
    # n = 0 with edges: reported as out of range
    s1 = torch.tensor([0], dtype=torch.int32, device="cuda")
    with torch.cuda.stream(stream):
        assert call_noalloc(contour, s1, s1, 0, labels, stats, stream) == contour.OK
    stream.synchronize()
    assert contour.read_stats(stats).status == contour.ERANGE
    # out-of-range ids are skipped and reported
    src = torch.tensor([0, 1, 9], dtype=torch.int32, device="cuda")
    dst = torch.tensor([1, 2, 3], dtype=torch.int32, device="cuda")
    with torch.cuda.stream(stream):
        assert call_noalloc(contour, src, dst, 5, labels, stats, stream, order="full") == contour.OK
    stream.synchronize()
    assert labels.tolist() == [0, 0, 0, 3, 4]
    assert contour.read_stats(stats).status == contour.ERANGE
    # the host-loop driver would allocate pinned memory: not offered
    assert call_noalloc(contour, src, dst, 5, labels, stats, stream, driver="hostloop") == contour.ENOTSUP
    # argument errors are synchronous
    assert lib.contour_cc_noalloc(None, None, -1, 4, None, None, None, None) == contour.EINVAL
    assert lib.contour_cc_noalloc(None, None, 3, 4, None, None, None, None) == contour.EINVAL
