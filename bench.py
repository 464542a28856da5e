#!/usr/bin/env python3
"""Benchmark: edges/s to exact connected-component labels on one MI355X.

One step = one full solve of the headline workload through the C ABI
(contour_cc_ex): edge grouping, label initialisation, every sweep of the
order-2 minimum mapping with the on-device convergence test, and the
statistics write.  Inputs are resident in HBM before the timed region starts.

Headline workload: R-MAT scale 24, edge factor 16 (a, b, c, d = 0.57, 0.19,
0.19, 0.05), vertex ids permuted, seed 1: n = 16,777,216, m = 268,435,456 --
the largest single-graph workload, whose edge stream (2.15 GB) is far larger
than the caches.

Printed: one JSON line with the throughput, a roofline object for the sweep
kernel (algorithmic bytes (8 + 8h) per edge-sweep divided by the kernel's
duration measured with events on its stream), the CPU oracle timed on the
host, and extras (the grid, the small ER graph, the batch of 20,000 graphs,
the serving trace, write-mode and operator comparisons, a cold-cache run and
the paper's own multicore CPU design).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "edges/s to exact CC labels (plain vs batched), HBM GB/s, p99 request latency"
HBM_PEAK_GBPS = 8000.0
WORKLOADS = ["rmat24_ef16", "grid4096_holes10", "er65536_m524288", "rmat24_ef16_share8"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_workload(name: str, seed: int):
    import graphgen
    if name == "grid4096_holes10":
        src, dst = graphgen.grid_holes(4096, 4096, 0.1, seed)
        return src, dst, 4096 * 4096
    if name == "rmat24_ef16":
        src, dst = graphgen.rmat(24, 16, seed)
        return src, dst, 1 << 24
    if name == "rmat24_ef16_share8":
        import numpy as np
        # one GPU's share of the R-MAT graph under the 1-D edge split of an
        # eight-GPU run: a seeded random eighth of the edges, all 2^24 labels
        src, dst = graphgen.rmat(24, 16, seed)
        keep = graphgen.share_mask(src.size, 8, 0, seed)
        return np.ascontiguousarray(src[keep]), np.ascontiguousarray(dst[keep]), 1 << 24
    if name == "er65536_m524288":
        src, dst = graphgen.er(65536, 524288, seed)
        return src, dst, 65536
    raise SystemExit("unknown workload %r" % name)


def order_value(order: str):
    return "full" if order == "full" else int(order)


def bytes_per_edge_sweep(order) -> int | None:
    # 8 bytes of edge ids streamed plus 2h label reads of 4 bytes (MM^h reads
    # L^1..L^h of both endpoints); chase-to-root has no fixed h.
    if order == "full":
        return None
    return 8 + 8 * int(order)


def time_gpu(contour, torch, s, d, n, steps, warmup, opts, cold_bytes=0):
    """Time `steps` solves back to back (events around each and around all),
    plus the sweep kernel of each through the library's timing hook.  With
    cold_bytes, a buffer of that size is written before each solve (outside
    its events) so the solve starts with the caches holding other data."""
    m = s.numel()
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    stats = [torch.zeros(4, dtype=torch.int32, device="cuda") for _ in range(steps)]

    def pair():
        return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    kev = [pair() for _ in range(steps)]
    sev = [pair() for _ in range(steps)]
    for a, b in kev:                       # create the underlying events
        a.record(stream)
        b.record(stream)
    lib = contour.load()
    o = contour.make_opts(**opts)
    scratch = torch.empty(cold_bytes // 4, dtype=torch.int32, device="cuda") if cold_bytes else None
    for _ in range(warmup):
        contour.cc_ex(s, d, n, labels=labels, stats=False, **opts)
    torch.cuda.synchronize()
    t0, t1 = pair()
    wall0 = time.perf_counter()
    t0.record(stream)
    for i in range(steps):
        if scratch is not None:
            scratch.fill_(i)
        lib.contour_set_timing_events(kev[i][0].cuda_event, kev[i][1].cuda_event)
        sev[i][0].record(stream)
        rc = lib.contour_cc_ex(ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(d.data_ptr()), m, n,
                               ctypes.c_void_p(labels.data_ptr()), ctypes.byref(o),
                               ctypes.c_void_p(stats[i].data_ptr()),
                               ctypes.c_void_p(stream.cuda_stream))
        sev[i][1].record(stream)
        if rc != 0:
            raise RuntimeError("contour_cc_ex failed: %d" % rc)
    t1.record(stream)
    torch.cuda.synchronize()
    wall1 = time.perf_counter()
    lib.contour_set_timing_events(None, None)
    return dict(total_ms=t0.elapsed_time(t1), wall_ms=(wall1 - wall0) * 1e3,
                step_ms=[a.elapsed_time(b) for a, b in sev], kernel_ms=[a.elapsed_time(b) for a, b in kev],
                stats=[x.tolist() for x in stats], labels=labels)


def source_hash() -> str:
    """Hash of the HIP sources and the C ABI header (names the kernel build)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2311_02811_amd", "csrc", "*")))
    files.append(os.path.join(ROOT, "include", "contour.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_figures(workload: str):
    """Counter figures of the sweep kernel from the committed rocprofv3
    summary, when it was taken on this workload with these exact sources:
    calibrated HBM bytes per launch and the L2 hit rate."""
    path = os.path.join(ROOT, "profiles", "k_persistent_%s.md" % workload)
    if not os.path.exists(path):
        return None
    import re
    text = open(path).read()
    h = re.search(r"csrc_sha256: ([0-9a-f]+)", text)
    if not h or h.group(1) != source_hash():
        return None
    out = {}
    t = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if t:
        out["traffic"] = int(t.group(1))
    l2 = re.search(r"l2_hit_rate: ([0-9.]+)", text)
    if l2:
        out["l2_hit_rate"] = float(l2.group(1))
    return out or None


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def roofline(order, m, r, figures, n=None):
    """Roofline object of the sweep kernel from a time_gpu result.  With n,
    also the compulsory-traffic rate: each sweep reads the edges once and the
    labels once and writes them once (8m + 8n bytes)."""
    bpe = bytes_per_edge_sweep(order)
    if bpe is None:
        return None
    sweeps = statistics.mean(x[1] for x in r["stats"])
    kernel_ms = statistics.mean(r["kernel_ms"])
    achieved = sweeps * m * bpe / (kernel_ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
            "kernel": "k_persistent", "kernel_ms": round(kernel_ms, 4),
            "bytes_per_edge_sweep": bpe, "edge_sweeps_per_launch": sweeps * m}
    if n is not None:
        comp = sweeps * (8.0 * m + 8.0 * n) / (kernel_ms / 1e3) / 1e9
        roof["compulsory_GBps"] = round(comp, 1)
        roof["compulsory_frac"] = round(comp / HBM_PEAK_GBPS, 4)
    if figures:
        if "traffic" in figures:
            roof["traffic"] = figures["traffic"]
            dram = figures["traffic"] / (kernel_ms / 1e3) / 1e9
            roof["dram_GBps"] = round(dram, 1)
            roof["dram_frac"] = round(dram / HBM_PEAK_GBPS, 4)
        if "l2_hit_rate" in figures:
            roof["l2_hit_rate"] = figures["l2_hit_rate"]
    return roof


def bench_merge(contour, torch, n=1 << 24, reps=20):
    """contour_merge_min, the combine step of the edge-split design, on two
    label states of n labels where the peer is smaller everywhere (every
    label is read twice and written once: 12 bytes per label)."""
    idx = torch.arange(n, dtype=torch.int32, device="cuda")
    peer = (idx // 2).contiguous()
    base = idx.clone()
    lab = torch.empty_like(idx)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    lowered = None
    for i in range(reps + 2):
        lab.copy_(base)
        if i >= 2:
            ev[i - 2][0].record(stream)
        lowered = contour.merge_min(peer, lab, stream=stream)
        if i >= 2:
            ev[i - 2][1].record(stream)
    torch.cuda.synchronize()
    ms = [a.elapsed_time(b) for a, b in ev]
    med = statistics.median(ms)
    gbps = 12.0 * n / (med / 1e3) / 1e9
    return {"n": n, "ms_median": round(med, 4), "ms_min": round(min(ms), 4),
            "lowered": int(lowered.item()), "exact": bool(torch.equal(lab, torch.minimum(base, peer))),
            "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": "k_merge_min",
                         "bytes_per_label": 12}}


def gather_ceilings(contour, torch, s, d, n, sweep_ms):
    """The sweep's memory access pattern without its arithmetic
    (contour_gather_ceiling) on the copy the default solve sweeps: edges
    only, edges + destination gathers, edges + both gathers; each the best of
    5.  sweep_ms is the measured sweep kernel time per sweep."""
    lib = contour.load()
    m = s.numel()
    ranges = n > (1 << 20) and m >= 4 * n
    gs, gd = contour.group_edges(s, d, n, ranges=ranges)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    labels = torch.arange(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    out = {"layout": "grouped by source block%s" % (", then destination range" if ranges else "")}
    for mode, key in ((0, "edges_ms"), (1, "edges_dst_gather_ms"), (2, "edges_both_gathers_ms")):
        ts = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            rc = lib.contour_gather_ceiling(ctypes.c_void_p(gs.data_ptr()), ctypes.c_void_p(gd.data_ptr()), m,
                                            ctypes.c_void_p(labels.data_ptr()), n, mode,
                                            ctypes.c_void_p(sink.data_ptr()), ctypes.c_void_p(stream.cuda_stream))
            b.record(stream)
            if rc != 0:
                raise RuntimeError("contour_gather_ceiling failed: %d" % rc)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        out[key] = round(min(ts), 4)
    out["edges_GBps"] = round(8.0 * m / (out["edges_ms"] / 1e3) / 1e9, 1)
    out["sweep_ms"] = round(sweep_ms, 4)
    out["sweep_over_dst_gather_ceiling"] = round(sweep_ms / out["edges_dst_gather_ms"], 3)
    del gs, gd
    return out


def full_order_roofline(contour, s, d, n, m, r):
    """Roofline of a chase-to-root solve: its algorithmic bytes are the edge
    stream (8 B per edge-sweep) plus 4 B per chain read, counted in one
    instrumented solve (contour_cc_count_reads); the timed solves r give the
    sweeps and the kernel time."""
    _, st, reads = contour.cc_count_reads(s, d, n, order="full")
    sw_c = contour.read_stats(st).sweeps_executed
    reads_per_edge_sweep = int(reads.item()) / float(m * max(sw_c, 1))
    sweeps = statistics.mean(x[1] for x in r["stats"])
    kernel_ms = statistics.mean(r["kernel_ms"])
    bpe = 8 + 4 * reads_per_edge_sweep
    achieved = sweeps * m * bpe / (kernel_ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": "k_persistent",
            "kernel_ms": round(kernel_ms, 4), "bytes_per_edge_sweep": round(bpe, 3),
            "chain_reads_per_edge_sweep": round(reads_per_edge_sweep, 4),
            "chain_reads_from": "one contour_cc_count_reads solve, %d sweeps" % sw_c}


def summary(r, m):
    sw = [x[1] for x in r["stats"]]
    mean = statistics.mean(r["step_ms"])
    return {"ms_mean": round(mean, 4), "ms_median": round(statistics.median(r["step_ms"]), 4),
            "ms_min": round(min(r["step_ms"]), 4), "edges_per_s": round(m / mean * 1e3, 1),
            "sweeps": {"min": min(sw), "max": max(sw), "mean": statistics.mean(sw)},
            "sweep_kernel_ms": round(statistics.mean(r["kernel_ms"]), 4)}


def bench_plain_extra(contour, torch, name, seed, steps, modes, exact=None):
    """The plain single-graph solve on another workload, several modes."""
    import numpy as np
    import oracle
    src, dst, n = make_workload(name, seed)
    m = int(src.size)
    if exact is None:
        exact = oracle.uf_labels(src, dst, n)
    s, d = torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda()
    out = {"n": n, "m": m}
    for key, opts in modes:
        r = time_gpu(contour, torch, s, d, n, steps, 1, opts)
        res = summary(r, m)
        res["exact"] = bool(np.array_equal(r["labels"].cpu().numpy(), exact))
        if not opts:
            res["roofline"] = roofline(2, m, r, profile_figures(name), n)
        elif opts == dict(order=3):
            res["roofline"] = roofline(3, m, r, None, n)
        elif opts == dict(order="full"):
            res["roofline"] = full_order_roofline(contour, s, d, n, m, r)
        out[key] = res
    return out, (src, dst, n, exact)


def bench_batched(contour, torch, seed, steps):
    """20,000 graphs in one plan launch vs one plain launch per graph (the
    20,000 contour_cc calls captured into one graph and replayed, so the
    baseline is the device's own time, not Python's call overhead)."""
    import numpy as np
    import graphgen
    import oracle
    b = graphgen.batch(20000, seed)
    exact = oracle.uf_batch(b.edge_off, b.vertex_off, b.src, b.dst)
    s = torch.from_numpy(b.src).cuda()
    d = torch.from_numpy(b.dst).cuda()
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def run_plan(tuning):
        plan = contour.BatchPlan(b.edge_off, b.vertex_off, s, d, tuning=tuning)
        plan.launch()
        torch.cuda.synchronize()
        t0.record(stream)
        for _ in range(steps):
            plan.launch()
        t1.record(stream)
        torch.cuda.synchronize()
        per_graph_sweeps = plan.stats[:, 1].cpu().numpy().astype(np.int64)
        res = (t0.elapsed_time(t1) / steps, plan.labels.cpu().numpy(), plan.classes(),
               float(per_graph_sweeps.mean()), per_graph_sweeps)
        plan.close()
        return res

    ms_default, batched_labels, classes, sweeps, gsweeps = run_plan(None)
    table = os.path.join(ROOT, "paper_2311_02811_amd", "tuning_gfx950.json")
    ms_tuned = None
    tuned_exact = True
    if os.path.exists(table):
        from paper_2311_02811_amd import autotune
        ms_tuned, tuned_labels, _, sweeps_tuned, gsweeps_tuned = run_plan(autotune.load_tuning(table))
        tuned_exact = bool(np.array_equal(tuned_labels, exact))
    ms = min(ms_default, ms_tuned) if ms_tuned else ms_default
    if ms_tuned and ms_tuned <= ms_default:
        sweeps, gsweeps = sweeps_tuned, gsweeps_tuned
    # baseline: one contour_cc per graph, same device-resident data, on a
    # side stream, captured once and replayed
    labels = torch.empty(int(b.vertex_off[-1]), dtype=torch.int32, device="cuda")
    lib = contour.load()
    eo, vo = b.edge_off, b.vertex_off
    sp, dp, lp = s.data_ptr(), d.data_ptr(), labels.data_ptr()
    side = torch.cuda.Stream()
    h = ctypes.c_void_p(side.cuda_stream)

    def per_graph():
        for g in range(b.num_graphs):
            rc = lib.contour_cc(ctypes.c_void_p(sp + 4 * int(eo[g])), ctypes.c_void_p(dp + 4 * int(eo[g])),
                                int(eo[g + 1] - eo[g]), int(vo[g + 1] - vo[g]),
                                ctypes.c_void_p(lp + 4 * int(vo[g])), h)
            if rc != 0:
                raise RuntimeError("contour_cc failed on graph %d: %d" % (g, rc))

    contour.reserve(int(b.m.max()), int(b.n.max()), stream=side)
    with torch.cuda.stream(side):
        per_graph()                       # eager once: the stream's workspace exists
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side, capture_error_mode="relaxed"):
        per_graph()
    labels.fill_(-1)
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    base_same = bool(np.array_equal(labels.cpu().numpy(), exact))
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(side)
    graph.replay()
    z.record(side)
    torch.cuda.synchronize()
    ms_base = a.elapsed_time(z)
    del graph
    G, M = b.num_graphs, int(b.m.sum())
    # roofline of the launch: edge-sweeps of every graph (its own sweep
    # count times its edges) at the order-2 count of 24 bytes each (a lower
    # bound where a class runs order 3 or chase-to-root), and the edge stream
    # alone (8 bytes per edge-sweep); the small graphs' labels sit in LDS or
    # the caches, so this is an algorithmic rate, not DRAM traffic
    edge_sweeps = int((gsweeps * b.m.astype(np.int64)).sum())
    alg = edge_sweeps * 24.0 / (ms / 1e3) / 1e9
    roof = {"bound": "hbm", "achieved": round(alg, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(alg / HBM_PEAK_GBPS, 4), "traffic": None, "kernel": "batched plan launch",
            "bytes_per_edge_sweep": 24, "edge_sweeps_per_launch": edge_sweeps,
            "edge_stream_GBps": round(edge_sweeps * 8.0 / (ms / 1e3) / 1e9, 1)}
    return {"graphs": G, "sum_n": int(b.n.sum()), "sum_m": M, "classes": classes, "roofline": roof,
            "ms_per_batch": round(ms, 3), "ms_per_batch_default": round(ms_default, 3),
            "ms_per_batch_tuned": round(ms_tuned, 3) if ms_tuned else None,
            "graphs_per_s": round(G / ms * 1e3, 1), "edges_per_s": round(M / ms * 1e3, 1),
            "sweeps_mean": round(sweeps, 3),
            "exact_vs_oracle": bool(np.array_equal(batched_labels, exact)) and tuned_exact,
            "per_graph_plain_ms": round(ms_base, 3),
            "per_graph_plain_graphs_per_s": round(G / ms_base * 1e3, 1),
            "per_graph_plain_exact": base_same,
            "per_graph_plain_how": "20,000 contour_cc calls captured into one hipGraph and replayed",
            "speedup_vs_per_graph": round(ms_base / ms, 2)}, (b, exact)


def bench_serving(contour, torch, seed, batch, batch_exact, seconds, rate, pool_big):
    """Poisson arrivals: the serving loop against FIFO plain launches, every
    result checked against the oracle; then the whole trace at once (load
    above what either can serve) for the saturated rates."""
    import numpy as np
    import graphgen
    import oracle
    big_pool, big_exact = [], []
    for k in range(pool_big):
        s2, d2 = graphgen.rmat(22, 16, seed + 100 + k)
        big_exact.append(torch.from_numpy(oracle.uf_labels(s2, d2, 1 << 22)))
        big_pool.append((torch.from_numpy(s2).pin_memory(), torch.from_numpy(d2).pin_memory(), 1 << 22))
    src_p = torch.from_numpy(batch.src).pin_memory()
    dst_p = torch.from_numpy(batch.dst).pin_memory()
    small_exact = torch.from_numpy(batch_exact)
    warm_s = 1.0
    count = int((seconds + warm_s) * rate)
    t_arr, big, pick = graphgen.poisson_trace(count, rate, 0.01, batch.num_graphs, len(big_pool), seed)

    def req(i):
        if big[i]:
            return big_pool[int(pick[i])]
        g = int(pick[i])
        a, b_ = int(batch.edge_off[g]), int(batch.edge_off[g + 1])
        return src_p[a:b_], dst_p[a:b_], int(batch.n[g])

    def expect(i):
        if big[i]:
            return big_exact[int(pick[i])]
        g = int(pick[i])
        return small_exact[int(batch.vertex_off[g]):int(batch.vertex_off[g + 1])]

    def check(outs):
        bad = 0
        for i in range(count):
            n_ = req(i)[2]
            if not torch.equal(outs[i][:n_], expect(i)):
                bad += 1
        return bad

    outs = [torch.empty(max(req(i)[2], 1), dtype=torch.int32).pin_memory() for i in range(count)]
    edges = sum(len(req(i)[0]) for i in range(count))

    def serve(paced):
        srv = contour.Server(lanes=4)
        for o in outs:
            o.fill_(-1)
        t_start = time.perf_counter() + 0.05
        ids = []
        for i in range(count):
            if paced:
                while time.perf_counter() < t_start + t_arr[i]:
                    pass
            s_, d_, n_ = req(i)
            ids.append(srv.submit(s_, d_, n_, outs[i]))
        srv.drain()
        res = {}
        while True:
            got = srv.poll(8192)
            if not got:
                break
            for r in got:
                res[r["id"]] = r
        srv.close()
        keep = [i for i in range(count) if not paced or t_arr[i] >= warm_s]
        lat = [(res[ids[i]]["t_done_ns"] - res[ids[i]]["t_submit_ns"]) / 1e6 for i in keep]
        t_first = min(res[i]["t_submit_ns"] for i in ids)
        t_last = max(res[i]["t_done_ns"] for i in ids)
        span = (t_last - t_first) / 1e9
        ok = all(res[i]["status"] == 0 for i in ids)
        return {"p50_ms": round(pct(lat, 50), 3), "p99_ms": round(pct(lat, 99), 3),
                "graphs_per_s": round(count / span, 1), "edges_per_s": round(edges / span, 1),
                "all_ok": ok, "wrong_vs_oracle": check(outs)}

    lib = contour.load()
    stream = torch.cuda.current_stream()
    h = ctypes.c_void_p(stream.cuda_stream)
    maxm = max(len(req(i)[0]) for i in range(count))
    maxn = max(req(i)[2] for i in range(count))
    ds = torch.empty(maxm, dtype=torch.int32, device="cuda")
    dd = torch.empty(maxm, dtype=torch.int32, device="cuda")
    dl = torch.empty(maxn, dtype=torch.int32, device="cuda")
    contour.reserve(maxm, maxn)

    def fifo(paced):
        for o in outs:
            o.fill_(-1)
        lat = []
        t0 = time.perf_counter() + 0.05
        for i in range(count):
            arrive = t0 + t_arr[i] if paced else time.perf_counter()
            while paced and time.perf_counter() < arrive:
                pass
            s_, d_, n_ = req(i)
            m_ = len(s_)
            if m_:
                ds[:m_].copy_(s_, non_blocking=True)
                dd[:m_].copy_(d_, non_blocking=True)
            rc = lib.contour_cc(ctypes.c_void_p(ds.data_ptr()), ctypes.c_void_p(dd.data_ptr()), m_, n_,
                                ctypes.c_void_p(dl.data_ptr()), h)
            if rc != 0:
                raise RuntimeError("contour_cc failed: %d" % rc)
            outs[i][:n_].copy_(dl[:n_], non_blocking=True)
            stream.synchronize()
            if not paced or t_arr[i] >= warm_s:
                lat.append((time.perf_counter() - arrive) * 1e3)
        span = time.perf_counter() - (t0 + t_arr[0] if paced else t0 - 0.05)
        return {"p50_ms": round(pct(lat, 50), 3), "p99_ms": round(pct(lat, 99), 3),
                "graphs_per_s": round(count / span, 1), "edges_per_s": round(edges / span, 1),
                "wrong_vs_oracle": check(outs)}

    out = {"requests": count, "rate_per_s": rate, "seconds": seconds, "warmup_seconds": warm_s,
           "big_requests": int(big.sum()), "big_pool": len(big_pool),
           "latency_excludes_warmup": True}
    log("serving: paced trace")
    out["served"] = serve(True)
    log("serving: FIFO plain, paced")
    out["fifo_plain"] = fifo(True)
    log("serving: whole trace at once")
    out["saturated_served"] = serve(False)
    log("serving: FIFO plain, back to back")
    out["saturated_fifo_plain"] = fifo(False)
    out["exact_vs_oracle"] = all(out[k]["wrong_vs_oracle"] == 0 for k in
                                 ("served", "fifo_plain", "saturated_served", "saturated_fifo_plain"))
    return out


def cpu_baseline(src, dst, n, budget_s):
    import oracle
    times = []
    labels = None
    t_end = time.perf_counter() + budget_s
    while True:
        t = time.perf_counter()
        labels = oracle.uf_labels(src, dst, n)
        times.append(time.perf_counter() - t)
        if time.perf_counter() >= t_end or len(times) >= 50:
            break
    return labels, times


def cpu_contour_omp(src, dst, n, exact, budget_s):
    """The paper's own multicore design (asynchronous, plain stores, early
    check; order 2) on all host threads, checked against the oracle."""
    import numpy as np
    import oracle
    times, sweeps, threads, same = [], [], 0, True
    t_end = time.perf_counter() + budget_s
    while True:
        t = time.perf_counter()
        lab, sw, threads = oracle.contour_omp(src, dst, n, 2)
        times.append(time.perf_counter() - t)
        sweeps.append(sw)
        same &= bool(np.array_equal(lab, exact))
        if time.perf_counter() >= t_end or len(times) >= 20:
            break
    t = statistics.median(times)
    return {"value": round(src.size / t, 1), "unit": "edges/s", "cores": threads,
            "nproc": os.cpu_count(), "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
            "kind": "paper's CPU design (OpenMP, asynchronous, plain stores, early check, order 2)",
            "runs": len(times), "median_s": round(t, 3), "sweeps": sweeps, "exact": same}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat24_ef16", choices=WORKLOADS)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--order", default="2")
    ap.add_argument("--write", default="plain", choices=["plain", "atomic"])
    ap.add_argument("--driver", default="persistent", choices=["persistent", "hostloop"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall-clock budget for each CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--reorder", default="auto", choices=["auto", "on", "off"])
    ap.add_argument("--dst-ranges", default="auto", help="auto, on, off or a range shift 16..30")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--edges-per-thread", type=int, default=0)
    ap.add_argument("--chunk-tiles", type=int, default=0)
    ap.add_argument("--max-sweeps", type=int, default=0,
                    help="stop each solve after this many sweeps (0: run to convergence); for profiling "
                         "the first sweeps on their own, the labels are then not final")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads, batched, serving, cold and A/B measurements")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-pool", type=int, default=8, help="R-MAT scale-22 graphs in the serving pool")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized int32 buffer --steps times (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2311_02811_amd as contour

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(args.steps):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": nbytes, "copies": args.steps}))
        return
    log("generating %s (seed %d)" % (args.workload, args.seed))
    src, dst, n = make_workload(args.workload, args.seed)
    m = int(src.size)
    order = order_value(args.order)
    dr = int(args.dst_ranges) if args.dst_ranges.isdigit() else args.dst_ranges
    opts = dict(order=order, write=args.write, driver=args.driver, reorder=args.reorder,
                block=args.block, edges_per_thread=args.edges_per_thread,
                chunk_tiles=args.chunk_tiles, dst_ranges=dr, max_sweeps=args.max_sweeps)
    s = torch.from_numpy(src).cuda()
    d = torch.from_numpy(dst).cuda()
    log("timing %d steps after %d warm-up steps: n=%d m=%d %r" % (args.steps, args.warmup, n, m, opts))
    r = time_gpu(contour, torch, s, d, n, args.steps, args.warmup, opts)
    ms_per_step = r["total_ms"] / args.steps
    sweeps = [x[1] for x in r["stats"]]
    status = sorted(set(x[0] for x in r["stats"]))
    value = m / (ms_per_step / 1e3)
    default_cfg = (args.reorder, args.block, args.edges_per_thread, args.chunk_tiles, args.write,
                   args.driver, args.order, args.dst_ranges, args.max_sweeps) == (
                       "auto", 0, 0, 0, "plain", "persistent", "2", "auto", 0)
    roof = roofline(order, m, r, profile_figures(args.workload) if default_cfg else None, n)
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_median": round(statistics.median(r["step_ms"]), 4),
        "ms_min": round(min(r["step_ms"]), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "seed": args.seed,
                   "order": order, "write": args.write, "driver": args.driver,
                   "reorder": args.reorder, "dst_ranges": args.dst_ranges, "block": args.block,
                   "edges_per_thread": args.edges_per_thread, "chunk_tiles": args.chunk_tiles,
                   "max_sweeps": args.max_sweeps},
        "sweeps": {"min": min(sweeps), "max": max(sweeps), "mean": statistics.mean(sweeps)},
        "status": status,
        "edge_sweeps_per_s": round(statistics.mean(sweeps) * m / (statistics.mean(r["kernel_ms"]) / 1e3), 1),
        "roofline": roof,
    }
    gpu_labels = r["labels"].cpu().numpy()
    r_kernel_ms = r["kernel_ms"]
    del r
    exact = None
    if not args.no_cpu_baseline:
        log("CPU oracle baseline (%.0f s budget)" % args.cpu_seconds)
        exact, times = cpu_baseline(src, dst, n, args.cpu_seconds)
        t = statistics.median(times)
        out["cpu_baseline"] = {"value": round(m / t, 1), "unit": "edges/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "sequential union-find on the whole workload graph, "
                                         "%d runs, median %.3f s" % (len(times), t)}
        out["exact"] = bool(np.array_equal(exact, gpu_labels))
    if not args.no_extras:
        import oracle
        if exact is None:
            exact = oracle.uf_labels(src, dst, n)
        extras = {}
        if not args.no_cpu_baseline:
            log("CPU: the paper's multicore design (%.0f s budget)" % args.cpu_seconds)
            extras["cpu_contour_omp"] = cpu_contour_omp(src, dst, n, exact, args.cpu_seconds)
        log("gather ceilings")
        sweep_ms = roof["kernel_ms"] / out["sweeps"]["mean"] if roof else statistics.mean(r_kernel_ms) / out["sweeps"]["mean"]
        extras["ceilings"] = gather_ceilings(contour, torch, s, d, n, sweep_ms)
        log("cold caches: 1 GiB written before each solve")
        rc = time_gpu(contour, torch, s, d, n, 5, 1, opts, cold_bytes=1 << 30)
        extras["cold"] = summary(rc, m)
        extras["cold"]["exact"] = bool(np.array_equal(rc["labels"].cpu().numpy(), exact))
        del rc
        log("modes on %s" % args.workload)
        modes = {}
        # operator choice (Section III-B-4): C-1, and the mixed schedules
        # C-11mm (order 1 for the first sweep) and C-1m1m, at order 2
        for key, o2 in (("order_3", dict(order=3)), ("order_full", dict(order="full")),
                        ("order_1", dict(order=1)), ("schedule_11mm", dict(schedule="11mm", k1=1)),
                        ("schedule_1m1m", dict(schedule="1m1m")),
                        ("dst_ranges_off", dict(dst_ranges="off")),
                        ("write_atomic", dict(write="atomic")),
                        ("hostloop_plain", dict(driver="hostloop")),
                        ("hostloop_atomic", dict(driver="hostloop", write="atomic"))):
            rr = time_gpu(contour, torch, s, d, n, 3, 1, o2)
            modes[key] = summary(rr, m)
            modes[key]["exact"] = bool(np.array_equal(rr["labels"].cpu().numpy(), exact))
            if key in ("order_3", "order_1"):
                modes[key]["roofline"] = roofline(int(key[-1]), m, rr, None)
            if key == "order_full":
                modes[key]["roofline"] = full_order_roofline(contour, s, d, n, m, rr)
            del rr
        extras[args.workload + "_modes"] = modes
        del s, d
        torch.cuda.empty_cache()
        for name in ("grid4096_holes10", "rmat24_ef16"):
            if name == args.workload:
                continue
            log("extra: %s" % name)
            extras[name], _ = bench_plain_extra(
                contour, torch, name, args.seed, 5,
                [("order_2", dict()), ("order_3", dict(order=3)), ("order_full", dict(order="full")),
                 ("schedule_11mm", dict(schedule="11mm", k1=1)), ("schedule_1m1m", dict(schedule="1m1m")),
                 ("hostloop_plain", dict(driver="hostloop")),
                 ("hostloop_atomic", dict(driver="hostloop", write="atomic"))])
            torch.cuda.empty_cache()
        log("extra: label merge of the edge-split design, n = 2^24")
        extras["merge_min_n16777216"] = bench_merge(contour, torch)
        log("extra: ER n=65536 m=524288")
        extras["er65536_m524288"], _ = bench_plain_extra(contour, torch, "er65536_m524288", args.seed, 20,
                                                         [("order_2", dict()), ("order_1", dict(order=1))])
        log("extra: batched 20,000 graphs")
        extras["batched20000"], (batch, batch_exact) = bench_batched(contour, torch, args.seed, 3)
        torch.cuda.empty_cache()
        log("extra: serving, Poisson 2000/s for %.1f s" % args.serve_seconds)
        extras["serving_poisson2000"] = bench_serving(contour, torch, args.seed, batch, batch_exact,
                                                      args.serve_seconds, 2000.0, args.serve_pool)
        out["extras"] = extras
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
