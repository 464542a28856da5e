"""ctypes view of libcontour.so (the C ABI declared in include/contour.h).

Only argument marshalling lives here: every step of the computation runs in
the HIP library.  There is no fallback: if the library is missing, loading
fails with an error.
"""
from __future__ import annotations

import ctypes
import os

from ._build import LIB_PATH

_lib = None

c_i32p = ctypes.POINTER(ctypes.c_int32)
c_i64p = ctypes.POINTER(ctypes.c_int64)


class ContourOpts(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int32) for name in (
        "order", "schedule", "k1", "write_mode", "update", "driver", "max_sweeps", "warm_start",
        "block", "edges_per_thread", "chunk_tiles", "grid", "reorder", "window", "dst_ranges")]


class ContourStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("sweeps_executed", ctypes.c_int32),
                ("sweeps_with_writes", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ContourBatch(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int32),
                ("h_edge_offsets", c_i64p),
                ("h_vertex_offsets", c_i64p),
                ("src", ctypes.c_void_p),
                ("dst", ctypes.c_void_p),
                ("labels_out", ctypes.c_void_p),
                ("stats_out", ctypes.c_void_p)]


class ClassTuning(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("block", ctypes.c_int32),
                ("edges_per_thread", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("cls", ClassTuning * 3), ("lds_max_vertices", ctypes.c_int32),
                ("wg_max_edges", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("lanes", ctypes.c_int32),
                ("batch_max", ctypes.c_int32), ("small_edges", ctypes.c_int64),
                ("opts", ContourOpts)]


class RequestResult(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32),
                ("sweeps_executed", ctypes.c_int32), ("t_submit_ns", ctypes.c_int64),
                ("t_admit_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64)]


# Exported symbols and their C signatures (restype, argtypes).
SIGNATURES = {
    "contour_default_opts": (None, [ctypes.POINTER(ContourOpts)]),
    "contour_cc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    "contour_cc_ex": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ContourOpts),
                                     ctypes.c_void_p, ctypes.c_void_p]),
    "contour_cc_add_edges": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ContourOpts),
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "contour_cc_count_reads": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                              ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ContourOpts),
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "contour_gather_ceiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "contour_merge_min": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                         ctypes.c_void_p]),
    "contour_reserve": (ctypes.c_int, [ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ContourOpts),
                                       ctypes.c_void_p]),
    "contour_cc_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ContourOpts),
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "contour_group_edges_ranges": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_void_p]),
    "contour_group_edges": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "contour_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "contour_last_hip_error": (ctypes.c_int, []),
    "contour_version": (ctypes.c_char_p, []),
    "contour_set_timing_events": (None, [ctypes.c_void_p, ctypes.c_void_p]),

    "contour_batch_plan_create": (ctypes.c_int, [ctypes.POINTER(ContourBatch),
                                                 ctypes.POINTER(ContourOpts),
                                                 ctypes.POINTER(ctypes.c_void_p)]),
    "contour_batch_plan_create_tuned": (ctypes.c_int, [ctypes.POINTER(ContourBatch),
                                                       ctypes.POINTER(ContourOpts),
                                                       ctypes.POINTER(BatchTuning),
                                                       ctypes.POINTER(ctypes.c_void_p)]),
    "contour_batch_plan_classes": (ctypes.c_int, [ctypes.c_void_p, c_i32p]),
    "contour_batch_plan_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "contour_batch_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "contour_cc_batched": (ctypes.c_int, [ctypes.POINTER(ContourBatch), ctypes.POINTER(ContourOpts),
                                          ctypes.c_void_p]),
    "contour_server_default_config": (None, [ctypes.POINTER(ServerConfig)]),
    "contour_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig),
                                             ctypes.POINTER(ctypes.c_void_p)]),
    "contour_server_submit": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                                             ctypes.POINTER(ctypes.c_int64)]),
    "contour_server_poll": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(RequestResult),
                                           ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32)]),
    "contour_server_drain": (ctypes.c_int, [ctypes.c_void_p]),
    "contour_server_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "contour_server_now_ns": (ctypes.c_int64, []),
}

OPTIONAL_SIGNATURES = {}


def lib_path() -> str:
    return LIB_PATH


def load():
    """Load libcontour.so, or raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcontour.so is not built (expected at %s); run "
                           "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in {**SIGNATURES, **OPTIONAL_SIGNATURES}.items():
        fn = getattr(lib, name, None)
        if fn is None:
            if name in SIGNATURES:
                raise RuntimeError("libcontour.so does not export %s" % name)
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
