"""CPU oracle for the Contour connectivity path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product library
never loads it, and it shares no code with the HIP path: its C part
(``cc_oracle.c``) and the Python models (``contour_model.py``) are written
from the paper alone.

Contents
  uf_labels / bfs_labels   the plain definition of the result (Sections II-A,
                           II-D): labels[v] = minimum vertex id of v's component,
                           by union-find and by breadth-first search.
  scipy_labels             the same through scipy's connected_components,
                           relabelled to minimum ids (a library route).
  uf_batch                 per-graph local labels of a CSR-of-graphs batch.
  check_labels             the invariants of a converged label array.
  contour_omp              the paper's own multicore CPU design (Algorithm 1,
                           asynchronous, early check, no atomics; Section
                           III-B) on all host threads: the timed CPU Contour
                           baseline, checked against uf_labels.
  contour_model            the algorithm itself (Def. 1-3, Alg. 1, the
                           asynchronous variant of Section III-B), for sweep
                           counts and per-iteration states.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_OMP_SRC = os.path.join(_HERE, "contour_omp.c")
_OMP_PATH = os.path.join(_HERE, "libcontour_omp.so")
_lib = None
_omp = None
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile cc_oracle.c (plain C, no OpenMP) into liboracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp,
                               _SRC])
        os.replace(tmp, _LIB_PATH)
    if force or not os.path.exists(_OMP_PATH):
        tmp = _OMP_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
                               "-o", tmp, _OMP_SRC])
        os.replace(tmp, _OMP_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    for name in ("oracle_uf_labels", "oracle_bfs_labels"):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [_i32p, _i32p, ctypes.c_int64, ctypes.c_int32, _i32p]
    lib.oracle_uf_batch.restype = ctypes.c_int
    lib.oracle_uf_batch.argtypes = [ctypes.c_int32, _i64p, _i64p, _i32p, _i32p, _i32p]
    lib.oracle_bfs_ecc.restype = ctypes.c_int64
    lib.oracle_bfs_ecc.argtypes = [_i32p, _i32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                   _i32p]
    _lib = lib
    return lib


def _as32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _call(fn, src, dst, n):
    src, dst = _as32(src), _as32(dst)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    labels = np.empty(max(n, 0), np.int32)
    rc = fn(src.ctypes.data_as(_i32p), dst.ctypes.data_as(_i32p), src.size, n,
            labels.ctypes.data_as(_i32p))
    if rc != 0:
        raise ValueError("oracle rejected the input (rc=%d): bad size or id outside [0, n)" % rc)
    return labels


def _load_omp():
    global _omp
    if _omp is not None:
        return _omp
    if not os.path.exists(_OMP_PATH):
        build(force=False)
    lib = ctypes.CDLL(_OMP_PATH)
    lib.contour_omp_cc.restype = ctypes.c_int
    lib.contour_omp_cc.argtypes = [_i32p, _i32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                   _i32p, _i32p, _i32p]
    _omp = lib
    return lib


def contour_omp(src, dst, n: int, order: int = 2):
    """The paper's CPU design of Contour on all OpenMP threads (MM^order,
    order 0 = chase to the root).  Returns (labels, sweeps, threads)."""
    src, dst = _as32(src), _as32(dst)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    labels = np.empty(max(n, 0), np.int32)
    sw, nt = ctypes.c_int32(0), ctypes.c_int32(0)
    rc = _load_omp().contour_omp_cc(src.ctypes.data_as(_i32p), dst.ctypes.data_as(_i32p), src.size, n,
                                    int(order), labels.ctypes.data_as(_i32p), ctypes.byref(sw),
                                    ctypes.byref(nt))
    if rc != 0:
        raise ValueError("contour_omp rejected the input (rc=%d)" % rc)
    return labels, int(sw.value), int(nt.value)


def uf_labels(src, dst, n: int) -> np.ndarray:
    """Minimum vertex id per component, by sequential union-find."""
    return _call(_load().oracle_uf_labels, src, dst, n)


def bfs_labels(src, dst, n: int) -> np.ndarray:
    """Minimum vertex id per component, by BFS from each vertex in increasing order."""
    return _call(_load().oracle_bfs_labels, src, dst, n)


def uf_batch(edge_off, vertex_off, src, dst) -> np.ndarray:
    eo = np.ascontiguousarray(edge_off, dtype=np.int64)
    vo = np.ascontiguousarray(vertex_off, dtype=np.int64)
    src, dst = _as32(src), _as32(dst)
    labels = np.empty(int(vo[-1]), np.int32)
    rc = _load().oracle_uf_batch(eo.size - 1, eo.ctypes.data_as(_i64p), vo.ctypes.data_as(_i64p),
                                 src.ctypes.data_as(_i32p), dst.ctypes.data_as(_i32p),
                                 labels.ctypes.data_as(_i32p))
    if rc != 0:
        raise ValueError("oracle rejected graph %d of the batch" % (-1 - rc))
    return labels


def bfs_ecc(src, dst, n: int, s: int):
    """(eccentricity of s, farthest vertex) by BFS."""
    src, dst = _as32(src), _as32(dst)
    far = ctypes.c_int32(0)
    ecc = _load().oracle_bfs_ecc(src.ctypes.data_as(_i32p), dst.ctypes.data_as(_i32p), src.size,
                                 n, s, ctypes.byref(far))
    if ecc < 0:
        raise ValueError("bad input for bfs_ecc")
    return int(ecc), int(far.value)


def diameter_lower_bound(src, dst, n: int, start: int = 0) -> int:
    """Double-sweep BFS lower bound on the diameter of start's component."""
    _, far = bfs_ecc(src, dst, n, start)
    ecc, _ = bfs_ecc(src, dst, n, far)
    return ecc


def scipy_labels(src, dst, n: int) -> np.ndarray:
    """Minimum vertex id per component through scipy.sparse.csgraph."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    src, dst = _as32(src), _as32(dst)
    if n == 0:
        return np.empty(0, np.int32)
    g = sp.coo_matrix((np.ones(src.size, np.int8), (src, dst)), shape=(n, n)).tocsr()
    _, comp = connected_components(g, directed=False)
    minv = np.full(comp.max() + 1, n, np.int64)
    np.minimum.at(minv, comp, np.arange(n, dtype=np.int64))
    return minv[comp].astype(np.int32)


def check_labels(src, dst, n: int, labels, n_components: int | None = None) -> list[str]:
    """Invariants of a converged label array; returns a list of violations.

    Endpoints of every edge carry equal labels; L[v] <= v; L[L[v]] = L[v]
    (every vertex points at a root: one star per component, Section II-A);
    the number of roots equals the number of components when that is given.
    """
    src, dst = _as32(src), _as32(dst)
    L = np.asarray(labels)
    bad = []
    if L.shape != (n,):
        return ["labels has shape %r, expected (%d,)" % (L.shape, n)]
    if n == 0:
        return bad
    if L.min() < 0 or L.max() >= n:
        return ["label outside [0, n)"]
    if src.size and np.any(L[src] != L[dst]):
        bad.append("an edge joins different labels")
    if np.any(L > np.arange(n)):
        bad.append("some L[v] > v")
    if np.any(L[L] != L):
        bad.append("some L[L[v]] != L[v]")
    if n_components is not None:
        roots = int(np.count_nonzero(L == np.arange(n)))
        if roots != n_components:
            bad.append("%d roots for %d components" % (roots, n_components))
    return bad
