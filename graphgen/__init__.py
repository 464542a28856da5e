"""Seeded synthetic graph generators (inputs only, no connectivity arithmetic).

The C library ``graphgen.c`` does the work; this module loads it with ctypes
and returns numpy int32 SoA edge arrays.  Every generator is a pure function
of its arguments and seed (counter-based SplitMix64 draws), independent of the
OpenMP thread count.

These inputs stand in for the paper's datasets (Section IV-A, Table I), which
are not available here: ER graphs for the small real-world graphs, a 2-D grid
with holes for the long-diameter road network, R-MAT for the power-law web and
social graphs, and a batch mix of many small graphs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile graphgen.c into libgraphgen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    lib.gg_mix64.restype = ctypes.c_uint64
    lib.gg_mix64.argtypes = [ctypes.c_uint64]
    lib.gg_draw.restype = ctypes.c_uint64
    lib.gg_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
    lib.gg_er.restype = ctypes.c_int64
    lib.gg_er.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, _i32p, _i32p]
    lib.gg_permutation.restype = ctypes.c_int
    lib.gg_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, _i32p]
    lib.gg_lattice_edges.restype = ctypes.c_int64
    lib.gg_lattice_edges.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
    lib.gg_grid_holes.restype = ctypes.c_int64
    lib.gg_grid_holes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.c_int, _i32p, _i32p]
    lib.gg_rmat.restype = ctypes.c_int64
    lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_uint64, ctypes.c_int, _i32p, _i32p]
    lib.gg_batch_sizes.restype = ctypes.c_int
    lib.gg_batch_sizes.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                   _i32p, _i64p, _i32p]
    lib.gg_batch_fill.restype = ctypes.c_int
    lib.gg_batch_fill.argtypes = [ctypes.c_int32, ctypes.c_uint64, _i32p, _i64p, _i32p, _i64p,
                                  _i32p, _i32p]
    lib.gg_poisson_trace.restype = ctypes.c_int
    lib.gg_poisson_trace.argtypes = [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, _f64p,
                                     _i32p, _i64p]
    lib.gg_shuffle_edges.restype = ctypes.c_int
    lib.gg_shuffle_edges.argtypes = [ctypes.c_int64, ctypes.c_uint64, _i32p, _i32p]
    lib.gg_num_threads.restype = ctypes.c_int
    lib.gg_num_threads.argtypes = []
    _lib = lib
    return lib


def _p32(a):
    return a.ctypes.data_as(_i32p)


def _p64(a):
    return a.ctypes.data_as(_i64p)


def mix64(z: int) -> int:
    return int(_load().gg_mix64(z & (2**64 - 1)))


def draw(seed: int, stream: int, i: int) -> int:
    return int(_load().gg_draw(seed, stream, i))


def num_threads() -> int:
    return int(_load().gg_num_threads())


def er(n: int, m: int, seed: int):
    """G(n, m): exactly m distinct undirected edges, no self-loops."""
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    got = _load().gg_er(n, m, seed, _p32(src), _p32(dst))
    if got != m:
        raise ValueError("gg_er failed for n=%d m=%d" % (n, m))
    return src, dst


def permutation(n: int, seed: int, stream: int = 4) -> np.ndarray:
    perm = np.empty(n, np.int32)
    _load().gg_permutation(n, seed, stream, _p32(perm))
    return perm


def lattice_edges(rows: int, cols: int, nv: int | None = None) -> int:
    nv = rows * cols if nv is None else nv
    return int(_load().gg_lattice_edges(rows, cols, nv))


def grid_holes(rows: int, cols: int, delete_frac: float, seed: int, permute_ids: bool = False):
    """rows x cols lattice, delete round(delete_frac * E) edges, random order."""
    total = lattice_edges(rows, cols)
    keep = total - int(round(delete_frac * total))
    src = np.empty(keep, np.int32)
    dst = np.empty(keep, np.int32)
    got = _load().gg_grid_holes(rows, cols, keep, seed, int(permute_ids), _p32(src), _p32(dst))
    if got != keep:
        raise ValueError("gg_grid_holes failed")
    return src, dst


def rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19, permute_ids=True):
    """R-MAT with m = edge_factor * 2**scale edges (self-loops and duplicates kept)."""
    m = edge_factor << scale
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    got = _load().gg_rmat(scale, m, a, b, c, seed, int(permute_ids), _p32(src), _p32(dst))
    if got != m:
        raise ValueError("gg_rmat failed")
    return src, dst


def share_mask(m: int, p: int, i: int, seed: int) -> np.ndarray:
    """Edges of share i when m edges are split into p seeded random shares
    (the 1-D edge split of a p-GPU run)."""
    return np.random.default_rng([seed, 0x5EED, p]).integers(0, p, m) == i


def shuffle_edges(src: np.ndarray, dst: np.ndarray, seed: int) -> None:
    assert src.dtype == np.int32 and dst.dtype == np.int32 and src.size == dst.size
    _load().gg_shuffle_edges(src.size, seed, _p32(src), _p32(dst))


@dataclass
class Batch:
    """A CSR-of-graphs batch: graph g owns vertices vertex_off[g]..vertex_off[g+1]
    (local ids 0..n_g-1) and edges edge_off[g]..edge_off[g+1] of src/dst."""
    n: np.ndarray          # int32 [G]
    m: np.ndarray          # int64 [G]
    kind: np.ndarray       # int32 [G], 0 = ER, 1 = grid with holes
    vertex_off: np.ndarray  # int64 [G+1]
    edge_off: np.ndarray    # int64 [G+1]
    src: np.ndarray        # int32 [sum m], local ids
    dst: np.ndarray

    @property
    def num_graphs(self) -> int:
        return int(self.n.size)

    def graph(self, g: int):
        a, b = int(self.edge_off[g]), int(self.edge_off[g + 1])
        return self.src[a:b], self.dst[a:b], int(self.n[g])


def batch_sizes(G: int, seed: int, median=2000.0, sigma=1.5, n_lo=64, n_hi=1 << 20,
                d_lo=2.0, d_hi=16.0):
    n = np.empty(G, np.int32)
    m = np.empty(G, np.int64)
    kind = np.empty(G, np.int32)
    _load().gg_batch_sizes(G, seed, median, sigma, n_lo, n_hi, d_lo, d_hi, _p32(n), _p64(m),
                           _p32(kind))
    return n, m, kind


def batch(G: int, seed: int, median=2000.0, sigma=1.5, n_lo=64, n_hi=1 << 20, d_lo=2.0,
          d_hi=16.0) -> Batch:
    n, m, kind = batch_sizes(G, seed, median, sigma, n_lo, n_hi, d_lo, d_hi)
    vo = np.zeros(G + 1, np.int64)
    eo = np.zeros(G + 1, np.int64)
    np.cumsum(n, out=vo[1:])
    np.cumsum(m, out=eo[1:])
    src = np.empty(int(eo[-1]), np.int32)
    dst = np.empty(int(eo[-1]), np.int32)
    rc = _load().gg_batch_fill(G, seed, _p32(n), _p64(m), _p32(kind), _p64(eo), _p32(src),
                               _p32(dst))
    if rc != 0:
        raise ValueError("gg_batch_fill failed")
    return Batch(n, m, kind, vo, eo, src, dst)


def poisson_trace(count: int, rate: float, p_big: float, pool_small: int, pool_big: int,
                  seed: int):
    t = np.empty(count, np.float64)
    big = np.empty(count, np.int32)
    pick = np.empty(count, np.int64)
    _load().gg_poisson_trace(count, rate, p_big, pool_small, pool_big, seed,
                             t.ctypes.data_as(_f64p), _p32(big), _p64(pick))
    return t, big, pick
