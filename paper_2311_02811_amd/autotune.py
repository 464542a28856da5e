"""Autotuner for batched plans: per size class, the operator order and the
launch geometry that solve a representative batch fastest.

The batch's graphs fall into three classes (include/contour.h): labels in LDS
with one workgroup per graph (0), labels in global memory with one workgroup
per graph (1), several workgroups per graph (2).  The operator order is free
per graph (every order reaches the same labels, Definition 3 and the Graph
Convergence theorem), and so is the geometry.  The tuner does a coordinate
search: for each class in turn it tries every candidate (order, block, edges
per thread) with the other classes held at their current best, times whole
plan launches, and keeps the fastest.  Every candidate's labels must equal the
first candidate's bit for bit, or the search stops with an error.

The result is a small JSON table keyed by the GPU architecture:

    {"arch": "gfx950", "classes": [{"order": 2, "block": 512, "edges_per_thread": 1}, ...],
     "lds_max_vertices": 0, "wg_max_edges": 0, "batch_ms": ...}

`load_tuning(path)` turns it back into a `contour_batch_tuning_t` for
`BatchPlan(..., tuning=...)`.
"""
from __future__ import annotations

import itertools
import json
import statistics

ORDERS = (2, 3, "full")
CLASS_CANDIDATES = {
    0: [dict(block=b, edges_per_thread=e) for b, e in itertools.product((256, 512, 1024), (1, 2))],
    1: [dict(block=b, edges_per_thread=e) for b, e in itertools.product((256, 512, 1024), (1, 2, 4))],
    2: [dict(block=b, edges_per_thread=e) for b, e in itertools.product((256, 512), (2, 4, 8))],
}


def candidates(cls: int, orders=ORDERS):
    """All (order, block, edges_per_thread) choices tried for a class."""
    return [dict(order=o, **g) for o in orders for g in CLASS_CANDIDATES[cls]]


def to_json(classes, lds_max_vertices=0, wg_max_edges=0, batch_ms=None, arch="gfx950") -> str:
    return json.dumps({"arch": arch, "classes": classes, "lds_max_vertices": lds_max_vertices,
                       "wg_max_edges": wg_max_edges, "batch_ms": batch_ms}, indent=1)


def from_json(text: str):
    d = json.loads(text)
    if not isinstance(d.get("classes"), list) or len(d["classes"]) != 3:
        raise ValueError("a tuning table has three classes")
    for c in d["classes"]:
        o = c.get("order", 0)
        if not (o in (0, "full", -1) or (isinstance(o, int) and 1 <= o <= 1024)):
            raise ValueError("bad order %r" % (o,))
        if c.get("block", 0) not in (0, 256, 512, 1024):
            raise ValueError("bad block %r" % (c.get("block"),))
        if c.get("edges_per_thread", 0) not in (0, 1, 2, 4, 8):
            raise ValueError("bad edges_per_thread %r" % (c.get("edges_per_thread"),))
    return d


def load_tuning(path: str):
    """Read a tuning table written by tune() as a BatchTuning structure."""
    from . import make_tuning
    with open(path) as f:
        d = from_json(f.read())
    return make_tuning(d["classes"], d.get("lds_max_vertices", 0), d.get("wg_max_edges", 0))


def _time_plan(contour, torch, batch_dev, spec, lds_max, wg_max, reps):
    eo, vo, s, d = batch_dev
    plan = contour.BatchPlan(eo, vo, s, d, tuning=contour.make_tuning(spec, lds_max, wg_max))
    try:
        plan.launch()
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            plan.launch()
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        return statistics.median(times), plan.labels.clone(), plan.classes()
    finally:
        plan.close()


def tune(edge_off, vertex_off, src, dst, reps=3, orders=ORDERS, lds_max_vertices=0, wg_max_edges=0,
         out_path=None, log=print):
    """Coordinate search over per-class settings on one batch (device int32
    tensors src/dst, host offsets).  Returns the JSON table (and writes it to
    out_path when given)."""
    import torch
    import paper_2311_02811_amd as contour
    batch_dev = (edge_off, vertex_off, src, dst)
    best = [dict(order=2), dict(order=2), dict(order=2)]
    best_ms, ref, classes = _time_plan(contour, torch, batch_dev, best, lds_max_vertices, wg_max_edges, reps)
    log("tune: start %.3f ms, classes %r" % (best_ms, classes))
    for cls in range(3):
        if classes[cls] == 0:
            continue
        for cand in candidates(cls, orders):
            spec = [dict(x) for x in best]
            spec[cls] = cand
            ms, labels, _ = _time_plan(contour, torch, batch_dev, spec, lds_max_vertices, wg_max_edges, reps)
            if not torch.equal(labels, ref):
                raise RuntimeError("tune: candidate %r changed the labels" % (spec,))
            if ms < best_ms:
                best_ms, best = ms, spec
                log("tune: class %d -> %r  %.3f ms" % (cls, cand, ms))
    table = to_json(best, lds_max_vertices, wg_max_edges, round(best_ms, 4))
    if out_path:
        with open(out_path, "w") as f:
            f.write(table + "\n")
    return table


def main(argv=None):
    """python -m paper_2311_02811_amd.autotune --out tuning.json [--graphs G --seed S]:
    tune on a seeded batch drawn like the 20,000-graph workload."""
    import argparse
    import sys
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import torch
    import graphgen
    ap = argparse.ArgumentParser(description="tune per-class settings of batched plans")
    ap.add_argument("--out", required=True)
    ap.add_argument("--graphs", type=int, default=20000)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args(argv)
    b = graphgen.batch(args.graphs, args.seed)
    s = torch.from_numpy(b.src).cuda()
    d = torch.from_numpy(b.dst).cuda()
    print(tune(b.edge_off, b.vertex_off, s, d, reps=args.reps, out_path=args.out,
               log=lambda *a: print(*a, flush=True)))


if __name__ == "__main__":
    main()
