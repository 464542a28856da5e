#!/usr/bin/env python3
"""Benchmark: edges/s to exact connected-component labels on one MI355X.

One step = one full solve of the headline workload through the C ABI
(contour_cc_ex): label initialisation, every sweep of the order-2 minimum
mapping with the on-device convergence test, and the statistics write.
Inputs are resident in HBM before the timed region starts.

Headline workload: 4096 x 4096 grid with 10% of its lattice edges deleted
(seed 1), edges in random order, n = 16,777,216, m = 30,191,616.

Printed: one JSON line with the throughput, a roofline object for the sweep
kernel (algorithmic bytes (8 + 8h) per edge-sweep divided by the kernel's
duration measured with events on its stream), and the CPU oracle timed on
the host for comparison.  Progress goes to stderr.
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


def time_gpu(contour, torch, src, dst, n, steps, warmup, opts):
    s = torch.from_numpy(src).cuda()
    d = torch.from_numpy(dst).cuda()
    m = src.size
    labels = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    stats = [torch.zeros(4, dtype=torch.int32, device="cuda") for _ in range(steps)]
    kev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    for a, b in kev:                       # create the underlying events
        a.record(stream)
        b.record(stream)
    lib = contour.load()
    o = contour.make_opts(**opts)
    for _ in range(warmup):
        contour.cc_ex(s, d, n, labels=labels, stats=False, **opts)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t0.record(stream)
    for i in range(steps):
        lib.contour_set_timing_events(kev[i][0].cuda_event, kev[i][1].cuda_event)
        rc = lib.contour_cc_ex(ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(d.data_ptr()), m, n,
                               ctypes.c_void_p(labels.data_ptr()), ctypes.byref(o),
                               ctypes.c_void_p(stats[i].data_ptr()),
                               ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError("contour_cc_ex failed: %d" % rc)
    t1.record(stream)
    torch.cuda.synchronize()
    wall1 = time.perf_counter()
    lib.contour_set_timing_events(None, None)
    total_ms = t0.elapsed_time(t1)
    kernel_ms = [a.elapsed_time(b) for a, b in kev]
    st = [x.tolist() for x in stats]
    return dict(total_ms=total_ms, wall_ms=(wall1 - wall0) * 1e3, kernel_ms=kernel_ms, stats=st,
                labels=labels.cpu().numpy())


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


def measured_traffic(workload: str):
    """HBM bytes per sweep-kernel launch from the committed rocprofv3 counter
    summary, when it was taken on this workload with these exact sources."""
    path = os.path.join(ROOT, "profiles", "k_persistent_%s.md" % {
        "grid4096_holes10": "grid4096_holes10"}.get(workload, workload))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    import re
    h = re.search(r"csrc_sha256: ([0-9a-f]+)", text)
    t = re.search(r"traffic_bytes_per_launch: (\d+)", text)
    if not h or not t or h.group(1) != source_hash():
        return None
    return int(t.group(1))


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def bench_plain_extra(contour, torch, name, seed, steps, orders):
    """Throughput of the plain single-graph solve on another workload."""
    src, dst, n = make_workload(name, seed)
    out = {"n": n, "m": int(src.size)}
    for order in orders:
        r = time_gpu(contour, torch, src, dst, n, steps, 1, dict(order=order))
        ms = r["total_ms"] / steps
        sw = [x[1] for x in r["stats"]]
        km = statistics.mean(r["kernel_ms"])
        key = "order_%s" % order
        out[key] = {"ms_per_solve": round(ms, 4), "edges_per_s": round(src.size / ms * 1e3, 1),
                    "sweeps_mean": statistics.mean(sw), "sweep_kernel_ms": round(km, 4)}
        bpe = bytes_per_edge_sweep(order)
        if bpe:
            out[key]["alg_GBps"] = round(statistics.mean(sw) * src.size * bpe / (km / 1e3) / 1e9, 1)
    return out


def bench_batched(contour, torch, seed, steps):
    """20,000 graphs in one plan launch vs one plain launch per graph."""
    import numpy as np
    import graphgen
    b = graphgen.batch(20000, seed)
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
        res = (t0.elapsed_time(t1) / steps, plan.labels.cpu().numpy(), plan.classes(),
               plan.stats[:, 1].float().mean().item())
        plan.close()
        return res

    ms_default, batched_labels, classes, sweeps = run_plan(None)
    table = os.path.join(ROOT, "paper_2311_02811_amd", "tuning_gfx950.json")
    ms_tuned = None
    if os.path.exists(table):
        from paper_2311_02811_amd import autotune
        ms_tuned, tuned_labels, _, _ = run_plan(autotune.load_tuning(table))
        if not np.array_equal(tuned_labels, batched_labels):
            raise RuntimeError("tuned plan changed the labels")
    ms = min(ms_default, ms_tuned) if ms_tuned else ms_default
    # baseline: one contour_cc per graph, same device-resident data, same stream
    labels = torch.empty(int(b.vertex_off[-1]), dtype=torch.int32, device="cuda")
    lib = contour.load()
    eo, vo = b.edge_off, b.vertex_off
    sp, dp, lp = s.data_ptr(), d.data_ptr(), labels.data_ptr()
    h = ctypes.c_void_p(stream.cuda_stream)
    wall0 = time.perf_counter()
    t0.record(stream)
    for g in range(b.num_graphs):
        lib.contour_cc(ctypes.c_void_p(sp + 4 * int(eo[g])), ctypes.c_void_p(dp + 4 * int(eo[g])),
                       int(eo[g + 1] - eo[g]), int(vo[g + 1] - vo[g]),
                       ctypes.c_void_p(lp + 4 * int(vo[g])), h)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_base = max(t0.elapsed_time(t1), wall * 1e3)
    same = bool(np.array_equal(labels.cpu().numpy(), batched_labels))
    G, M = b.num_graphs, int(b.m.sum())
    return {"graphs": G, "sum_n": int(b.n.sum()), "sum_m": M, "classes": classes,
            "ms_per_batch": round(ms, 3), "ms_per_batch_default": round(ms_default, 3),
            "ms_per_batch_tuned": round(ms_tuned, 3) if ms_tuned else None, "graphs_per_s": round(G / ms * 1e3, 1),
            "edges_per_s": round(M / ms * 1e3, 1), "sweeps_mean": round(sweeps, 3),
            "per_graph_plain_ms": round(ms_base, 3),
            "per_graph_plain_graphs_per_s": round(G / ms_base * 1e3, 1),
            "speedup_vs_per_graph": round(ms_base / ms, 2), "identical_labels": same}, b


def bench_serving(contour, torch, seed, batch, seconds, rate):
    """Poisson arrivals: micro-batched serving loop vs FIFO plain launches."""
    import numpy as np
    import graphgen
    big_pool = []
    for k in range(2):
        s2, d2 = graphgen.rmat(22, 16, seed + 100 + k)
        big_pool.append((torch.from_numpy(s2).pin_memory(), torch.from_numpy(d2).pin_memory(), 1 << 22))
    src_p = torch.from_numpy(batch.src).pin_memory()
    dst_p = torch.from_numpy(batch.dst).pin_memory()
    count = int(seconds * rate)
    t_arr, big, pick = graphgen.poisson_trace(count, rate, 0.01, batch.num_graphs, len(big_pool), seed)

    def req(i):
        if big[i]:
            return big_pool[int(pick[i])]
        g = int(pick[i])
        a, b_ = int(batch.edge_off[g]), int(batch.edge_off[g + 1])
        return src_p[a:b_], dst_p[a:b_], int(batch.n[g])

    outs = [torch.empty(max(req(i)[2], 1), dtype=torch.int32).pin_memory() for i in range(count)]
    # served
    srv = contour.Server(lanes=4)
    t_start = time.perf_counter() + 0.05
    ids = []
    for i in range(count):
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
    lat = [(res[i]["t_done_ns"] - res[i]["t_submit_ns"]) / 1e6 for i in ids]
    t_first = min(res[i]["t_submit_ns"] for i in ids)
    t_last = max(res[i]["t_done_ns"] for i in ids)
    span = (t_last - t_first) / 1e9
    edges = sum(len(req(i)[0]) for i in range(count))
    ok = all(res[i]["status"] == 0 for i in ids)
    # FIFO baseline: one plain solve per request in arrival order
    lib = contour.load()
    stream = torch.cuda.current_stream()
    h = ctypes.c_void_p(stream.cuda_stream)
    maxm = max(len(req(i)[0]) for i in range(count))
    maxn = max(req(i)[2] for i in range(count))
    ds = torch.empty(maxm, dtype=torch.int32, device="cuda")
    dd = torch.empty(maxm, dtype=torch.int32, device="cuda")
    dl = torch.empty(maxn, dtype=torch.int32, device="cuda")
    base_out = [torch.empty_like(o) for o in outs]
    lat_b = []
    same = True
    t0 = time.perf_counter() + 0.05
    for i in range(count):
        arrive = t0 + t_arr[i]
        while time.perf_counter() < arrive:
            pass
        s_, d_, n_ = req(i)
        m_ = len(s_)
        if m_:
            ds[:m_].copy_(s_, non_blocking=True)
            dd[:m_].copy_(d_, non_blocking=True)
        lib.contour_cc(ctypes.c_void_p(ds.data_ptr()), ctypes.c_void_p(dd.data_ptr()), m_, n_,
                       ctypes.c_void_p(dl.data_ptr()), h)
        base_out[i][:n_].copy_(dl[:n_], non_blocking=True)
        stream.synchronize()
        lat_b.append((time.perf_counter() - arrive) * 1e3)
    span_b = time.perf_counter() - t0 - t_arr[0]
    for i in range(0, count, max(1, count // 200)):
        n_ = req(i)[2]
        same &= bool(torch.equal(outs[i][:n_], base_out[i][:n_]))
    return {"requests": count, "rate_per_s": rate, "seconds": seconds, "big_requests": int(big.sum()),
            "all_ok": ok, "identical_to_plain": same,
            "served": {"p50_ms": round(pct(lat, 50), 3), "p99_ms": round(pct(lat, 99), 3),
                       "graphs_per_s": round(count / span, 1), "edges_per_s": round(edges / span, 1)},
            "fifo_plain": {"p50_ms": round(pct(lat_b, 50), 3), "p99_ms": round(pct(lat_b, 99), 3),
                           "graphs_per_s": round(count / span_b, 1),
                           "edges_per_s": round(edges / span_b, 1)}}


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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid4096_holes10",
                    choices=["grid4096_holes10", "rmat24_ef16", "er65536_m524288", "rmat24_ef16_share8"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--order", default="2")
    ap.add_argument("--write", default="plain", choices=["plain", "atomic"])
    ap.add_argument("--driver", default="persistent", choices=["persistent", "hostloop"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="wall-clock budget for the CPU oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--reorder", default="auto", choices=["auto", "on", "off"])
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--edges-per-thread", type=int, default=0)
    ap.add_argument("--chunk-tiles", type=int, default=0)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the R-MAT, ER, batched and serving measurements")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized int32 buffer --steps times (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
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
    opts = dict(order=order, write=args.write, driver=args.driver, reorder=args.reorder,
                block=args.block, edges_per_thread=args.edges_per_thread,
                chunk_tiles=args.chunk_tiles)
    log("timing %d steps after %d warm-up steps: n=%d m=%d %r" % (args.steps, args.warmup, n, m, opts))
    r = time_gpu(contour, torch, src, dst, n, args.steps, args.warmup, opts)
    ms_per_step = r["total_ms"] / args.steps
    sweeps = [s[1] for s in r["stats"]]
    status = sorted(set(s[0] for s in r["stats"]))
    kernel_ms = statistics.mean(r["kernel_ms"])
    value = m / (ms_per_step / 1e3)
    bpe = bytes_per_edge_sweep(order)
    roof = None
    if bpe is not None:
        alg_bytes = statistics.mean(sweeps) * m * bpe
        achieved = alg_bytes / (kernel_ms / 1e3) / 1e9
        default_cfg = (args.reorder, args.block, args.edges_per_thread, args.chunk_tiles, args.write,
                       args.driver, args.order) == ("auto", 0, 0, 0, "plain", "persistent", "2")
        traffic = measured_traffic(args.workload) if default_cfg else None
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "k_persistent" if args.driver == "persistent" else "k_sweep",
                "kernel_ms": round(kernel_ms, 4),
                "bytes_per_edge_sweep": bpe, "edge_sweeps_per_launch": statistics.mean(sweeps) * m}
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "seed": args.seed,
                   "order": order, "write": args.write, "driver": args.driver,
                   "reorder": args.reorder, "block": args.block,
                   "edges_per_thread": args.edges_per_thread, "chunk_tiles": args.chunk_tiles},
        "sweeps": {"min": min(sweeps), "max": max(sweeps), "mean": statistics.mean(sweeps)},
        "status": status,
        "edge_sweeps_per_s": round(statistics.mean(sweeps) * m / (kernel_ms / 1e3), 1),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("CPU oracle baseline (%.0f s budget)" % args.cpu_seconds)
        lab, times = cpu_baseline(src, dst, n, args.cpu_seconds)
        t = statistics.median(times)
        out["cpu_baseline"] = {"value": round(m / t, 1), "unit": "edges/s", "cores": 1,
                               "kind": "oracle",
                               "sample": "sequential union-find on the whole workload graph, "
                                         "%d runs, median %.3f s" % (len(times), t)}
        out["exact"] = bool(np.array_equal(lab, r["labels"]))
    if not args.no_extras:
        extras = {}
        log("extra: R-MAT scale 24")
        extras["rmat24_ef16"] = bench_plain_extra(contour, torch, "rmat24_ef16", args.seed, 3,
                                                  [2, 3, "full"])
        log("extra: ER n=65536 m=524288")
        extras["er65536_m524288"] = bench_plain_extra(contour, torch, "er65536_m524288", args.seed,
                                                      20, [2, 1])
        log("extra: batched 20,000 graphs")
        extras["batched20000"], batch = bench_batched(contour, torch, args.seed, 3)
        log("extra: serving, Poisson 2000/s for %.1f s" % args.serve_seconds)
        extras["serving_poisson2000"] = bench_serving(contour, torch, args.seed, batch,
                                                      args.serve_seconds, 2000.0)
        out["extras"] = extras
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
