"""Exact connected components on MI355X by the Contour minimum-mapping algorithm.

Python binding of libcontour.so (C ABI in include/contour.h).  PyTorch only
supplies device memory and streams; every step of the solve runs in the HIP
library, and there is no CPU fallback.

    labels = cc(src, dst, n)            # src, dst: int32 CUDA tensors
    labels[v] == min vertex id of v's component

Operator orders, schedules, write modes and drivers follow Definition 3,
Algorithm 1 and Section III-B of the paper (arXiv 2311.02811).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

from ._lib import (BatchTuning, ContourBatch, ContourOpts, RequestResult, ServerConfig,  # noqa: F401
                   load, lib_path)

ORDER_FULL = -1
_SCHED = {"fixed": 0, "11mm": 1, "1m1m": 2}
_WRITE = {"plain": 0, "atomic": 1}
_UPDATE = {"async": 0, "sync": 1}
_DRIVER = {"persistent": 0, "hostloop": 1}
_REORDER = {"auto": 0, "off": 1, "on": 2}

OK, EINVAL, ERANGE, ENOMEM, EHIP, ENOCONV, ENOTSUP, ETOOBIG = range(8)


class ContourError(RuntimeError):
    def __init__(self, code: int, what: str):
        lib = load()
        msg = lib.contour_status_string(code).decode()
        if code == EHIP:
            msg += " (hipError %d)" % lib.contour_last_hip_error()
        super().__init__("%s: %s" % (what, msg))
        self.code = code


@dataclass
class Stats:
    status: int
    sweeps_executed: int
    sweeps_with_writes: int


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check_edges(src, dst):
    torch = _torch()
    for name, t in (("src", src), ("dst", dst)):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or not t.is_cuda:
            raise TypeError("%s must be an int32 CUDA tensor" % name)
        if not t.is_contiguous():
            raise ValueError("%s must be contiguous" % name)
    if src.shape != dst.shape or src.dim() != 1:
        raise ValueError("src and dst must be 1-D of equal length")
    if src.device != dst.device:
        raise ValueError("src and dst are on different devices")


def make_opts(order=0, schedule="fixed", k1=2, write="plain", update="async",
              driver="persistent", max_sweeps=0, warm_start=False, block=0,
              edges_per_thread=0, chunk_tiles=0, grid=0, reorder="auto", window=0,
              dst_ranges="auto") -> ContourOpts:
    o = ContourOpts()
    load().contour_default_opts(ctypes.byref(o))
    o.order = ORDER_FULL if order in ("full", ORDER_FULL) else int(order)
    o.schedule = _SCHED[schedule]
    o.k1 = int(k1)
    o.write_mode = _WRITE[write]
    o.update = _UPDATE[update]
    o.driver = _DRIVER[driver]
    o.max_sweeps = int(max_sweeps)
    o.warm_start = 1 if warm_start else 0
    o.block = int(block)
    o.edges_per_thread = int(edges_per_thread)
    o.chunk_tiles = int(chunk_tiles)
    o.grid = int(grid)
    o.reorder = _REORDER[reorder]
    o.window = int(window)
    o.dst_ranges = int(dst_ranges) if isinstance(dst_ranges, int) else _REORDER[dst_ranges]
    return o


def cc(src, dst, n: int, labels=None, stream=None):
    """labels[v] = minimum vertex id of v's component (defaults: order 2,
    asynchronous update, plain stores, persistent driver)."""
    torch = _torch()
    _check_edges(src, dst)
    if labels is None:
        labels = torch.empty(max(int(n), 0), dtype=torch.int32, device=src.device)
    rc = load().contour_cc(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                           src.numel(), int(n), ctypes.c_void_p(labels.data_ptr()),
                           _stream_ptr(stream))
    if rc != OK:
        raise ContourError(rc, "contour_cc")
    return labels


def cc_ex(src, dst, n: int, labels=None, stream=None, stats: bool = True, **opts):
    """contour_cc_ex with keyword options (see make_opts).  Returns
    (labels, stats_tensor) where stats_tensor is a device int32[4]
    (status, sweeps_executed, sweeps_with_writes, 0); read_stats() converts it."""
    torch = _torch()
    _check_edges(src, dst)
    if labels is None:
        labels = torch.empty(max(int(n), 0), dtype=torch.int32, device=src.device)
    elif labels.dtype != torch.int32 or not labels.is_cuda or labels.numel() != n:
        raise ValueError("labels must be an int32 CUDA tensor of n elements")
    o = make_opts(**opts)
    st = torch.zeros(4, dtype=torch.int32, device=src.device) if stats else None
    rc = load().contour_cc_ex(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                              src.numel(), int(n), ctypes.c_void_p(labels.data_ptr()),
                              ctypes.byref(o), ctypes.c_void_p(st.data_ptr() if stats else 0),
                              _stream_ptr(stream))
    if rc != OK:
        raise ContourError(rc, "contour_cc_ex")
    return labels, st


def cc_count_reads(src, dst, n: int, labels=None, stream=None, **opts):
    """contour_cc_count_reads: (labels, stats_tensor, reads_tensor) where
    reads_tensor is a device int64[1] holding the label reads of the chains
    of every sweep run with an order above 3 or chase-to-root."""
    torch = _torch()
    _check_edges(src, dst)
    if labels is None:
        labels = torch.empty(max(int(n), 0), dtype=torch.int32, device=src.device)
    o = make_opts(**opts)
    st = torch.zeros(4, dtype=torch.int32, device=src.device)
    reads = torch.zeros(1, dtype=torch.int64, device=src.device)
    rc = load().contour_cc_count_reads(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                       src.numel(), int(n), ctypes.c_void_p(labels.data_ptr()),
                                       ctypes.byref(o), ctypes.c_void_p(st.data_ptr()),
                                       ctypes.c_void_p(reads.data_ptr()), _stream_ptr(stream))
    if rc != OK:
        raise ContourError(rc, "contour_cc_count_reads")
    return labels, st, reads


def reserve(m: int, n: int, stream=None, **opts):
    """contour_reserve: allocate the stream's workspace for graphs of up to m
    edges and n vertices, so that later solves on the stream within these
    sizes only enqueue kernels (and can be captured into a graph)."""
    o = make_opts(**opts)
    rc = load().contour_reserve(int(m), int(n), ctypes.byref(o), _stream_ptr(stream))
    if rc != OK:
        raise ContourError(rc, "contour_reserve")


def cc_noalloc(src, dst, n: int, labels, stats, stream=None, **opts):
    """contour_cc_noalloc: as cc_ex, but the library allocates nothing (its
    scratch is a fixed device array shared by every call on the device).
    `labels` (int32[n]) and `stats` (int32[4] or None) are caller-owned CUDA
    tensors; the call only enqueues work."""
    _check_edges(src, dst)
    o = make_opts(**opts)
    rc = load().contour_cc_noalloc(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                   src.numel(), int(n), ctypes.c_void_p(labels.data_ptr()),
                                   ctypes.byref(o), ctypes.c_void_p(stats.data_ptr() if stats is not None else 0),
                                   _stream_ptr(stream))
    if rc != OK:
        raise ContourError(rc, "contour_cc_noalloc")
    return labels, stats


def group_edges(src, dst, n: int, stream=None, ranges: bool = False):
    """contour_group_edges (or, with ranges=True, contour_group_edges_ranges):
    (src_out, dst_out), the edge list grouped as a reordering solve prepares
    it (stream ordered)."""
    torch = _torch()
    _check_edges(src, dst)
    so, do = torch.empty_like(src), torch.empty_like(dst)
    lib = load()
    fn = lib.contour_group_edges_ranges if ranges else lib.contour_group_edges
    rc = fn(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.numel(), int(n),
            ctypes.c_void_p(so.data_ptr()), ctypes.c_void_p(do.data_ptr()), _stream_ptr(stream))
    if rc != OK:
        raise ContourError(rc, "contour_group_edges_ranges" if ranges else "contour_group_edges")
    return so, do


def merge_min(peer, labels, stream=None, count: bool = True):
    """contour_merge_min: labels = min(labels, peer) elementwise, in place
    (stream ordered).  Returns a device int32 tensor of one element holding
    the number of labels lowered, or None with count=False."""
    torch = _torch()
    for t in (peer, labels):
        if t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("peer and labels must be contiguous int32 CUDA tensors")
    if peer.numel() != labels.numel():
        raise ValueError("peer and labels must have the same length")
    lowered = torch.empty(1, dtype=torch.int32, device=labels.device) if count else None
    rc = load().contour_merge_min(ctypes.c_void_p(peer.data_ptr()), ctypes.c_void_p(labels.data_ptr()),
                                  labels.numel(), ctypes.c_void_p(lowered.data_ptr() if count else 0),
                                  _stream_ptr(stream))
    if rc != OK:
        raise ContourError(rc, "contour_merge_min")
    return lowered


def add_edges(src, dst, n: int, labels, stream=None, stats: bool = True, **opts):
    """contour_cc_add_edges: `labels` (int32 CUDA tensor of n) holds the exact
    labels of a graph; after the call (stream ordered) it holds the labels of
    that graph plus the edges (src, dst).  Returns (labels, stats_tensor)."""
    torch = _torch()
    _check_edges(src, dst)
    if labels.dtype != torch.int32 or not labels.is_cuda or labels.numel() != n:
        raise ValueError("labels must be an int32 CUDA tensor of n elements")
    o = make_opts(**opts)
    st = torch.zeros(4, dtype=torch.int32, device=labels.device) if stats else None
    rc = load().contour_cc_add_edges(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                     src.numel(), int(n), ctypes.c_void_p(labels.data_ptr()),
                                     ctypes.byref(o), ctypes.c_void_p(st.data_ptr() if stats else 0),
                                     _stream_ptr(stream))
    if rc != OK:
        raise ContourError(rc, "contour_cc_add_edges")
    return labels, st


class Graph:
    """A graph on n vertices whose connected components are kept current on
    the device as edges arrive (a front end over contour_cc_add_edges).

        g = Graph(n)
        g.add_edges(src, dst)        # int32 CUDA tensors
        g.labels                     # labels[v] = minimum id of v's component
        g.num_components(), g.connected(u, v)
    """

    def __init__(self, n: int, device="cuda", **opts):
        torch = _torch()
        self.n = int(n)
        self.opts = opts
        self.labels = torch.arange(self.n, dtype=torch.int32, device=device)
        self.num_edges = 0

    def add_edges(self, src, dst, stream=None):
        _, st = add_edges(src, dst, self.n, self.labels, stream=stream, **self.opts)
        self.num_edges += src.numel()
        return read_stats(st)

    def num_components(self) -> int:
        torch = _torch()
        ids = torch.arange(self.n, dtype=torch.int32, device=self.labels.device)
        return int((self.labels == ids).sum().item())

    def connected(self, u: int, v: int) -> bool:
        return bool(self.labels[int(u)].item() == self.labels[int(v)].item())


def read_stats(st) -> Stats:
    v = st.tolist()
    return Stats(v[0], v[1], v[2])


def version() -> str:
    return load().contour_version().decode()


def make_tuning(classes=None, lds_max_vertices=0, wg_max_edges=0) -> BatchTuning:
    """Per-class choices for a batched plan: classes is a list of up to three
    dicts with keys order / block / edges_per_thread (0 or missing = auto)."""
    t = BatchTuning()
    for c, spec in enumerate(classes or []):
        if spec is None:
            continue
        o = spec.get("order", 0)
        t.cls[c].order = ORDER_FULL if o in ("full", ORDER_FULL) else int(o)
        t.cls[c].block = int(spec.get("block", 0))
        t.cls[c].edges_per_thread = int(spec.get("edges_per_thread", 0))
    t.lds_max_vertices = int(lds_max_vertices)
    t.wg_max_edges = int(wg_max_edges)
    return t


class BatchPlan:
    """A reusable plan that solves every graph of a CSR-of-graphs batch.

    edge_off, vertex_off: host int64 sequences of length G+1; src, dst: int32
    CUDA tensors of local ids; labels: int32 CUDA tensor of vertex_off[G]
    elements (allocated when None).  launch() enqueues one solve on a stream;
    the plan keeps references to the tensors it was built on.
    """

    def __init__(self, edge_off, vertex_off, src, dst, labels=None, stats=True, tuning=None,
                 **opts):
        import numpy as np
        torch = _torch()
        _check_edges(src, dst)
        self.edge_off = np.ascontiguousarray(edge_off, dtype=np.int64)
        self.vertex_off = np.ascontiguousarray(vertex_off, dtype=np.int64)
        self.num_graphs = self.edge_off.size - 1
        total_n = int(self.vertex_off[-1]) if self.num_graphs > 0 else 0
        if int(self.edge_off[-1] if self.num_graphs > 0 else 0) != src.numel():
            raise ValueError("edge_off[-1] must equal the number of edges")
        self.src, self.dst = src, dst
        self.labels = labels if labels is not None else torch.empty(
            max(total_n, 0), dtype=torch.int32, device=src.device)
        self.stats = torch.zeros((max(self.num_graphs, 1), 4), dtype=torch.int32,
                                 device=src.device) if stats else None
        b = ContourBatch()
        b.num_graphs = self.num_graphs
        b.h_edge_offsets = self.edge_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        b.h_vertex_offsets = self.vertex_off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        b.src = src.data_ptr()
        b.dst = dst.data_ptr()
        b.labels_out = self.labels.data_ptr()
        b.stats_out = self.stats.data_ptr() if stats else None
        self._batch = b
        self._opts = make_opts(**opts)
        self._tuning = tuning
        h = ctypes.c_void_p()
        lib = load()
        if tuning is not None:
            rc = lib.contour_batch_plan_create_tuned(ctypes.byref(b), ctypes.byref(self._opts),
                                                     ctypes.byref(tuning), ctypes.byref(h))
        else:
            rc = lib.contour_batch_plan_create(ctypes.byref(b), ctypes.byref(self._opts),
                                               ctypes.byref(h))
        if rc != OK:
            raise ContourError(rc, "contour_batch_plan_create")
        self._h = h

    def classes(self):
        counts = (ctypes.c_int32 * 3)()
        load().contour_batch_plan_classes(self._h, counts)
        return list(counts)

    def launch(self, stream=None):
        rc = load().contour_batch_plan_launch(self._h, _stream_ptr(stream))
        if rc != OK:
            raise ContourError(rc, "contour_batch_plan_launch")
        return self.labels

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().contour_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cc_batched(edge_off, vertex_off, src, dst, labels=None, stream=None, **opts):
    """Solve every graph of a batch once (create, launch and destroy a plan)."""
    plan = BatchPlan(edge_off, vertex_off, src, dst, labels=labels, **opts)
    try:
        plan.launch(stream)
        _torch().cuda.synchronize()
        return plan.labels, plan.stats
    finally:
        plan.close()


class Server:
    """Serving loop of contour_serve.h: submit host graphs as they arrive,
    poll finished requests.  Host arrays should be pinned (torch tensors with
    pin_memory=True, or any buffer from hipHostMalloc); the caller keeps each
    request's arrays alive until it is reported done."""

    def __init__(self, hbm_budget_bytes=0, lanes=0, batch_max=0, small_edges=0, **opts):
        lib = load()
        c = ServerConfig()
        lib.contour_server_default_config(ctypes.byref(c))
        c.hbm_budget_bytes = int(hbm_budget_bytes)
        c.lanes = int(lanes)
        c.batch_max = int(batch_max)
        c.small_edges = int(small_edges)
        c.opts = make_opts(**opts)
        h = ctypes.c_void_p()
        rc = lib.contour_server_create(ctypes.byref(c), ctypes.byref(h))
        if rc != OK:
            raise ContourError(rc, "contour_server_create")
        self._h = h
        self._keep = {}

    @staticmethod
    def now_ns() -> int:
        return int(load().contour_server_now_ns())

    def submit(self, src, dst, n: int, labels) -> int:
        """src, dst: host int32 tensors (or numpy arrays) of m ids; labels:
        host int32 buffer of n entries, written when the request is done."""
        def ptr(a):
            if a is None:
                return None
            if hasattr(a, "data_ptr"):
                return a.data_ptr()
            return a.ctypes.data
        rid = ctypes.c_int64()
        m = len(src)
        rc = load().contour_server_submit(self._h, ptr(src) if m else None,
                                          ptr(dst) if m else None, m, int(n),
                                          ptr(labels) if n else None, ctypes.byref(rid))
        if rc != OK:
            raise ContourError(rc, "contour_server_submit")
        self._keep[rid.value] = (src, dst, labels)
        return rid.value

    def poll(self, max_results=1024, wait_us=0):
        buf = (RequestResult * max(int(max_results), 1))()
        cnt = ctypes.c_int32()
        rc = load().contour_server_poll(self._h, buf, int(max_results), int(wait_us),
                                        ctypes.byref(cnt))
        if rc != OK:
            raise ContourError(rc, "contour_server_poll")
        out = []
        for i in range(cnt.value):
            r = buf[i]
            self._keep.pop(r.id, None)
            out.append(dict(id=r.id, status=r.status, sweeps=r.sweeps_executed,
                            t_submit_ns=r.t_submit_ns, t_admit_ns=r.t_admit_ns,
                            t_done_ns=r.t_done_ns))
        return out

    def drain(self):
        rc = load().contour_server_drain(self._h)
        if rc != OK:
            raise ContourError(rc, "contour_server_drain")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().contour_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
