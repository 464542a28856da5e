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
                    choices=["grid4096_holes10", "rmat24_ef16", "er65536_m524288"])
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
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
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
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
