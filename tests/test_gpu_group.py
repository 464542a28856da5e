"""GPU: grouping of the edge list by source block (contour_group_edges), the
copy a reordering solve sweeps.

The grouping is index work, so it is checked bit for bit against its
definition in the header: the same (src, dst) pairs, ordered by source block
and, within a block, by input chunk of 8192 edges.  The order inside one
(block, chunk) run is left free, so each run is compared as a multiset, and
every position's run is fixed.
"""
import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CHUNK = 8192


@pytest.fixture(scope="module")
def contour():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_2311_02811_amd as contour
    contour.load()
    return contour


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def expected_runs(src, n):
    """Run id (block, chunk) of every input edge and the stable order of the
    grouped copy, from the header's definition."""
    shift = 0
    while ((n - 1) >> shift) >= 1024:
        shift += 1
    k = ((n - 1) >> shift) + 1
    block = np.minimum(src.view(np.uint32) >> shift, k - 1).astype(np.int64)
    chunk = np.arange(src.size, dtype=np.int64) // CHUNK
    nch = (src.size + CHUNK - 1) // CHUNK
    run = block * nch + chunk
    order = np.argsort(run, kind="stable")
    return run[order], order


def check_grouping(contour, src, dst, n):
    print("group_edges n=%d m=%d" % (n, src.size), flush=True)
    so, do = contour.group_edges(dev(src), dev(dst), n)
    torch.cuda.synchronize()
    got_s, got_d = so.cpu().numpy(), do.cpu().numpy()
    run, order = expected_runs(src, n)
    exp_s, exp_d = src[order], dst[order]
    # pairs as one 64-bit key; within each run (fixed positions) compare the
    # multisets by sorting on (run, pair)
    def keyed(s, d):
        pair = (s.astype(np.int64) << 32) | d.view(np.uint32).astype(np.int64)
        return pair[np.lexsort((pair, run))]
    assert np.array_equal(keyed(got_s, got_d), keyed(exp_s, exp_d))


@pytest.mark.parametrize("n,m,seed", [
    (1 << 20, 2_500_003, 1),      # 1024 blocks, several chunk groups, ragged last chunk
    (1000, 70_001, 2),            # shift 0, K = 1000
    (1, 5, 3),                    # one block
    (3_000_001, 1_048_576 + 8192 * 3 + 1, 4),  # K < 1024 with shift 12, group boundary
    (77, 8192, 5),                # exactly one chunk
])
def test_grouping_matches_definition(contour, n, m, seed):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m, dtype=np.int64).astype(np.int32)
    dst = rng.integers(0, n, m, dtype=np.int64).astype(np.int32)
    check_grouping(contour, src, dst, n)


def test_grouping_of_ids_outside_range(contour):
    # ids outside [0, n) are moved unchanged into the last block
    rng = np.random.default_rng(6)
    n, m = 50_000, 100_000
    src = rng.integers(0, n, m, dtype=np.int64).astype(np.int32)
    dst = rng.integers(0, n, m, dtype=np.int64).astype(np.int32)
    src[::97] = -5
    src[3::101] = n + 7
    dst[5::89] = -(1 << 31)
    check_grouping(contour, src, dst, n)


def test_grouping_of_skewed_blocks(contour):
    # R-MAT degrees: a few blocks hold most of the edges
    src, dst = graphgen.rmat(18, 16, 7)
    check_grouping(contour, src, dst, 1 << 18)


def test_grouping_full_grid(contour):
    # the 4096 x 4096 grid with 10% holes, the size a solve reorders
    src, dst = graphgen.grid_holes(4096, 4096, 0.1, 1)
    check_grouping(contour, src, dst, 4096 * 4096)


def test_grouping_empty_is_a_no_op(contour):
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    so, do = contour.group_edges(e, e, 10)
    assert so.numel() == 0 and do.numel() == 0


# ------------------------------------------------------------------------
# contour_group_edges_ranges: the source-block grouping followed by a stable
# grouping by destination range.  Expected order from the header's
# definition: by range, then source block, then input chunk; the order inside
# one (range, block, chunk) run is free.

def expected_runs_ranges(src, dst, n):
    shift = 0
    while ((n - 1) >> shift) >= 1024:
        shift += 1
    k = ((n - 1) >> shift) + 1
    t = 19
    while ((n - 1) >> t) >= 64:
        t += 1
    r = ((n - 1) >> t) + 1
    block = np.minimum(src.view(np.uint32) >> shift, k - 1).astype(np.int64)
    rng_ = np.minimum(dst.view(np.uint32) >> t, r - 1).astype(np.int64)
    chunk = np.arange(src.size, dtype=np.int64) // CHUNK
    nch = (src.size + CHUNK - 1) // CHUNK
    run = (rng_ * k + block) * nch + chunk
    order = np.argsort(run, kind="stable")
    return run[order], order


def check_grouping_ranges(contour, src, dst, n):
    print("group_edges_ranges n=%d m=%d" % (n, src.size), flush=True)
    so, do = contour.group_edges(dev(src), dev(dst), n, ranges=True)
    torch.cuda.synchronize()
    got_s, got_d = so.cpu().numpy(), do.cpu().numpy()
    run, order = expected_runs_ranges(src, dst, n)
    exp_s, exp_d = src[order], dst[order]

    def keyed(s, d):
        pair = (s.astype(np.int64) << 32) | d.view(np.uint32).astype(np.int64)
        return pair[np.lexsort((pair, run))]
    assert np.array_equal(keyed(got_s, got_d), keyed(exp_s, exp_d))


@pytest.mark.parametrize("n,m,seed", [
    ((1 << 19) + 1, 300_001, 11),           # two ranges, the second one id wide
    (1 << 24, 3_000_017, 12),               # 32 ranges, ragged last chunk
    ((1 << 25) + 3, 2_000_000, 13),         # shift 20: 33 ranges -> t grows until < 64
    ((1 << 31) - 1, 500_000, 14),           # the largest n: 64 ranges of 2^25 ids
])
def test_grouping_by_ranges_matches_definition(contour, n, m, seed):
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m, dtype=np.int64).astype(np.int32)
    dst = rng.integers(0, n, m, dtype=np.int64).astype(np.int32)
    check_grouping_ranges(contour, src, dst, n)


def test_grouping_by_ranges_rmat_and_out_of_range(contour):
    src, dst = graphgen.rmat(21, 16, 15)
    n = 1 << 21
    src[::97] = -5
    dst[3::101] = n + 7
    dst[5::89] = -(1 << 31)
    check_grouping_ranges(contour, src, dst, n)


def test_grouping_by_ranges_argument_errors(contour):
    lib = contour.load()
    import ctypes
    p = ctypes.c_void_p(16)
    assert lib.contour_group_edges_ranges(p, p, 3, 1 << 19, p, p, None) == contour.EINVAL
    assert lib.contour_group_edges_ranges(p, p, -1, 1 << 20, p, p, None) == contour.EINVAL
    assert lib.contour_group_edges_ranges(None, None, 0, 1 << 20, None, None, None) == contour.OK
