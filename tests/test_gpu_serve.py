"""GPU tests of the serving loop (include/contour_serve.h).

Every request's labels must be bit-identical to the CPU oracle and to a
standalone solve of the same graph, whatever else is in flight: the result
of a request does not depend on the mix it was served in (tolerance 0,
labels are integers with a unique correct answer).
"""
import time

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


def pinned(a):
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32))
    return t.pin_memory()


def make_requests(seed, count, big_every=0):
    b = graphgen.batch(count, seed, median=800, sigma=1.4, n_lo=1, n_hi=60000)
    reqs = []
    for g in range(b.num_graphs):
        s, d, n = b.graph(g)
        reqs.append((s.copy(), d.copy(), n))
        if big_every and g % big_every == 0:
            s2, d2 = graphgen.rmat(16, 6, seed + g)
            reqs.append((s2, d2, 1 << 16))
    return reqs


def serve(contour, reqs, pace_s=0.0, **cfg):
    srv = contour.Server(**cfg)
    outs, ids = [], []
    for s, d, n in reqs:
        lab = torch.full((max(n, 1),), -7, dtype=torch.int32).pin_memory()
        ids.append(srv.submit(pinned(s), pinned(d), n, lab))
        outs.append(lab)
        if pace_s:
            time.sleep(pace_s)
    srv.drain()
    results = {}
    while True:
        got = srv.poll(4096)
        if not got:
            break
        for r in got:
            results[r["id"]] = r
    srv.close()
    return ids, outs, results


def test_serving_mix_matches_oracle_and_standalone(contour):
    reqs = make_requests(3, 300, big_every=60)
    print("requests", len(reqs), flush=True)
    ids, outs, results = serve(contour, reqs, lanes=4, small_edges=50000)
    assert len(results) == len(reqs)
    for (s, d, n), rid, lab in zip(reqs, ids, outs):
        r = results[rid]
        assert r["status"] == 0, r
        exp = oracle.uf_labels(s, d, n)
        assert np.array_equal(lab.numpy()[:n], exp), rid
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_done_ns"]
    # the same request alone, through the plain single-graph call
    for k in range(0, len(reqs), 23):
        s, d, n = reqs[k]
        if n == 0:
            continue
        alone = contour.cc(torch.from_numpy(s).cuda(), torch.from_numpy(d).cuda(), n).cpu().numpy()
        assert np.array_equal(alone, outs[k].numpy()[:n])


def test_serving_paced_arrivals_and_one_lane(contour):
    reqs = make_requests(5, 120, big_every=40)
    ids, outs, results = serve(contour, reqs, pace_s=0.0005, lanes=1, batch_max=16,
                               small_edges=30000)
    for (s, d, n), rid, lab in zip(reqs, ids, outs):
        assert results[rid]["status"] == 0
        assert np.array_equal(lab.numpy()[:n], oracle.uf_labels(s, d, n))


def test_serving_tight_budget_queues_and_rejects_oversize(contour):
    reqs = make_requests(7, 60)
    big_s, big_d = graphgen.rmat(18, 16, 1)                # ~33 MB of edges
    reqs.append((big_s, big_d, 1 << 18))
    # 8 MiB budget: small requests queue for memory; the big one can never fit
    ids, outs, results = serve(contour, reqs, hbm_budget_bytes=8 << 20, lanes=3)
    for (s, d, n), rid, lab in zip(reqs, ids, outs):
        r = results[rid]
        if n == 1 << 18:
            assert r["status"] == contour.ENOMEM
        else:
            assert r["status"] == 0
            assert np.array_equal(lab.numpy()[:n], oracle.uf_labels(s, d, n))


def test_serving_edge_cases(contour):
    e = np.zeros(0, np.int32)
    reqs = [(e, e, 0), (e, e, 5), (np.array([2], np.int32), np.array([2], np.int32), 3),
            (np.array([0, 9], np.int32), np.array([1, 1], np.int32), 4)]
    ids, outs, results = serve(contour, reqs)
    assert results[ids[0]]["status"] == 0
    assert np.array_equal(outs[1].numpy(), np.arange(5))
    assert np.array_equal(outs[2].numpy(), [0, 1, 2])
    assert results[ids[3]]["status"] == contour.ERANGE
    assert np.array_equal(outs[3].numpy(), [0, 0, 2, 3])


def test_serving_config5_trace_with_rmat22_matches_oracle(contour):
    # The serving workload's shape at full request size: Poisson arrivals at
    # 2000/s drawn from the batch distribution plus 1% R-MAT scale-22 graphs
    # (n = 4,194,304, m = 67,108,864) from a pool of two; one second of the
    # trace, paced, then the same requests all at once.  Every request is
    # compared with the oracle's labels of its pool item.
    b = graphgen.batch(2000, 11)
    small_exact = oracle.uf_batch(b.edge_off, b.vertex_off, b.src, b.dst)
    pool = []
    for k in range(2):
        s2, d2 = graphgen.rmat(22, 16, 500 + k)
        pool.append((pinned(s2), pinned(d2), 1 << 22, oracle.uf_labels(s2, d2, 1 << 22)))
    src_p, dst_p = pinned(b.src), pinned(b.dst)
    count = 2000
    t_arr, big, pick = graphgen.poisson_trace(count, 2000.0, 0.01, b.num_graphs, len(pool), 11)
    assert 5 <= int(big.sum()) <= 60

    def req(i):
        if big[i]:
            s, d, n, exp = pool[int(pick[i])]
            return s, d, n, exp
        g = int(pick[i])
        a, z = int(b.edge_off[g]), int(b.edge_off[g + 1])
        v0, v1 = int(b.vertex_off[g]), int(b.vertex_off[g + 1])
        return src_p[a:z], dst_p[a:z], v1 - v0, small_exact[v0:v1]

    for paced in (True, False):
        print("config-5 trace: %d requests (%d R-MAT-22), paced=%s" % (count, int(big.sum()), paced), flush=True)
        srv = contour.Server(lanes=4)
        outs, ids = [], []
        t0 = time.perf_counter()
        for i in range(count):
            if paced:
                while time.perf_counter() < t0 + t_arr[i]:
                    pass
            s, d, n, _ = req(i)
            lab = torch.full((max(n, 1),), -7, dtype=torch.int32).pin_memory()
            ids.append(srv.submit(s, d, n, lab))
            outs.append(lab)
        srv.drain()
        results = {}
        while True:
            got = srv.poll(4096)
            if not got:
                break
            for r in got:
                results[r["id"]] = r
        srv.close()
        assert len(results) == count
        for i in range(count):
            _, _, n, exp = req(i)
            assert results[ids[i]]["status"] == 0, i
            assert np.array_equal(outs[i].numpy()[:n], exp), (i, bool(big[i]))
