"""CPU models of the Contour algorithm itself (TEST INFRASTRUCTURE ONLY).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It is written from the paper and shares nothing with the
HIP library.

Notation follows Section II-B:
  * L is the label array, L^1[x] = L[x] and L^h[x] = L[L^{h-1}[x]];
  * the h-order minimum-mapping operator MM^h on an edge <w, v> (Definition 3)
    takes z^h = min(L^h[w], L^h[v]) and applies the conditional assignment of
    Definition 1 (x := z wherever x > z) to the entries at
    w, v, L[w], L[v], ..., L^{h-1}[w], L^{h-1}[v];
  * order 0 here means "chase to the root": follow L until L[x] = x and treat
    every vertex on the way, root included, as a target (the paper's C-m uses
    a large finite order, m = 1024, which behaves the same once every chain is
    shorter than m).

Models
  contour_sync    Algorithm 1 (C-Syn): every edge reads the old array L and
                  writes the update array L_u; the conditional assignments are
                  the compare-and-swap loop of Eq. (cas), i.e. an atomic
                  minimum, so one iteration is deterministic:
                  L_u[x] = min(L[x], min of z over all edge targets equal to x).
                  Iterations repeat while any label changes; the count includes
                  the last iteration that changes nothing.
  contour_async   Section III-B-1: one array updated in place, edges taken
                  sequentially in a given order, with the early convergence
                  check of Section III-B-2 evaluated on the values each edge
                  read before its own writes.
  contour_lost_update
                  the asynchronous update with plain (non-atomic) stores of
                  Section III-B-3, modelled as groups of edges that all read
                  first and then store in a shuffled order, last store wins.
  sharded_rounds  the multi-GPU design (not in the paper, one GPU is built):
                  the edge list split into shares, each share solved with
                  Algorithm 1's loop started from the current labels, the
                  shares' results combined by an elementwise minimum, rounds
                  repeated until one changes nothing.
Operator schedules (Section III-B-4): C-1, C-2, C-m, C-11mm, C-1m1m.

Loops are plain Python except in contour_sync, which uses numpy fancy indexing
and np.minimum.at for the per-iteration minimum; use small graphs.
"""
from __future__ import annotations

import math
import random
from typing import Callable, Sequence

import numpy as np

FULL = 0


# ------------------------------------------------------------ schedules --

def schedule(name: str, m: int = 1024, k1: int = 2) -> Callable[[int], int]:
    """Order used in iteration s (0-based) for the variants of Section III-B-4.

    C-1 / C-2: fixed order 1 / 2.  C-m: fixed order m.  C-11mm: order 1 for
    the first k1 iterations ("a few"), then order m.  C-1m1m: alternates order
    1 and order m, starting with 1.  Order 0 stands for chase-to-root.
    """
    if name == "C-1":
        return lambda s: 1
    if name == "C-2":
        return lambda s: 2
    if name == "C-3":
        return lambda s: 3
    if name == "C-m":
        return lambda s: m
    if name == "C-full":
        return lambda s: FULL
    if name == "C-11mm":
        return lambda s: 1 if s < k1 else m
    if name == "C-1m1m":
        return lambda s: 1 if s % 2 == 0 else m
    raise ValueError("unknown schedule %r" % name)


def theorem_bound(d_max: int) -> int:
    """Iteration bound of the Graph Convergence theorem: ceil(log_{3/2} d_max) + 1."""
    if d_max <= 1:
        return 1
    return int(math.ceil(math.log(d_max) / math.log(1.5) - 1e-12)) + 1


# ------------------------------------------------------ synchronous model --

def _levels(L: np.ndarray, x: np.ndarray, order: int) -> list[np.ndarray]:
    """[x, L[x], L^2[x], ...]: order+1 levels, or for order 0 until every chain
    has reached its root (the last level then repeats the roots)."""
    levels = [x]
    steps = 0
    while True:
        nxt = L[levels[-1]]
        levels.append(nxt)
        steps += 1
        settled = np.array_equal(nxt, levels[-2])
        if order == FULL:
            if settled:
                return levels
        elif steps == order or settled:
            # once every chain sits at a root, deeper levels only repeat it
            return levels


def sync_iteration(L: np.ndarray, src: np.ndarray, dst: np.ndarray, order: int) -> np.ndarray:
    """One iteration of Algorithm 1 with MM^order: returns L_u."""
    Lu = L.copy()
    m = src.size
    if m == 0:
        return Lu
    x = np.concatenate([src, dst]).astype(np.int64)
    lev = _levels(L, x, order)
    top = lev[-1]
    z = np.minimum(top[:m], top[m:])
    zz = np.concatenate([z, z])
    for t in lev[:-1]:
        np.minimum.at(Lu, t, zz)
    return Lu


def contour_sync(src, dst, n: int, sched: Callable[[int], int] | int = 2,
                 max_iter: int = 1 << 20, record: bool = False):
    """Algorithm 1 (C-Syn).  Returns (labels, iterations, changing, states).

    iterations counts every pass of the do-while loop including the final one
    that changes nothing; changing = iterations - 1 when converged.  states is
    the list of L after each iteration when record is set.
    """
    if isinstance(sched, int):
        fixed = sched
        sched = lambda s: fixed  # noqa: E731
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    L = np.arange(n, dtype=np.int64)
    states = []
    it = 0
    while it < max_iter:
        Lu = sync_iteration(L, src, dst, sched(it))
        it += 1
        changed = not np.array_equal(Lu, L)
        L = Lu
        if record:
            states.append(L.astype(np.int32))
        if not changed:
            return L.astype(np.int32), it, it - 1, states
    raise RuntimeError("no convergence within %d iterations" % max_iter)


# ----------------------------------------------------- asynchronous model --

def _chain(L: list, x: int, order: int) -> list:
    """[x, L[x], ..., L^order[x]] read from the current array (order 0: up to
    and including the first repeat of the root)."""
    c = [x]
    while True:
        y = L[c[-1]]
        c.append(y)
        if y == c[-2]:
            return c
        if order != FULL and len(c) == order + 1:
            return c


def mm_edge_reads(L: list, w: int, v: int, order: int):
    """Reads of MM^order on <w, v>: (targets, values read at them, z).

    targets[i] is written with z when the value read there exceeds z; the
    value read at target x_i is x_{i+1}, the next vertex of its chain.
    """
    cw, cv = _chain(L, w, order), _chain(L, v, order)
    z = min(cw[-1], cv[-1])
    targets = cw[:-1] + cv[:-1]
    values = cw[1:] + cv[1:]
    return targets, values, z


def contour_async(src, dst, n: int, sched: Callable[[int], int] | int = 2,
                  edge_order: Sequence[int] | None = None, max_sweeps: int = 1 << 20,
                  L0: Sequence[int] | None = None):
    """Asynchronous Contour (Section III-B-1) with the early convergence check.

    Each edge reads its chains, decides from those pre-write reads whether it
    changes anything (for order >= 2 this is exactly the paper's test
    L[v] != L^2[v] or L[w] != L^2[w] or L[v] != L[w]), then applies the
    conditional assignments in place.  A sweep in which no edge has anything
    to change ends the run.  Returns (labels, sweeps) where sweeps counts the
    final sweep that changed nothing.  L0 warm-starts from a label array that
    satisfies L0[x] <= x and lies in x's component.
    """
    if isinstance(sched, int):
        fixed = sched
        sched = lambda s: fixed  # noqa: E731
    src = [int(a) for a in src]
    dst = [int(b) for b in dst]
    order_idx = list(range(len(src))) if edge_order is None else list(edge_order)
    L = list(range(n)) if L0 is None else [int(a) for a in L0]
    for s in range(max_sweeps):
        h = sched(s)
        active = False
        for e in order_idx:
            targets, values, z = mm_edge_reads(L, src[e], dst[e], h)
            if any(val > z for val in values):
                active = True
            for x in targets:
                if L[x] > z:
                    L[x] = z
        if not active:
            return np.asarray(L, np.int32), s + 1
    raise RuntimeError("no convergence within %d sweeps" % max_sweeps)


def paper_check(L: list, w: int, v: int) -> bool:
    """The early-convergence predicate of Section III-B-2 for one edge."""
    return L[v] != L[L[v]] or L[w] != L[L[w]] or L[v] != L[w]


def contour_lost_update(src, dst, n: int, order: int = 2, group: int = 8, seed: int = 0,
                        max_sweeps: int = 1 << 20, record: bool = False):
    """Asynchronous Contour with plain stores and lost updates.

    Edges are processed in groups: every edge of a group reads its chains from
    the current array, then all their stores (z into each target whose read
    value exceeded z) are applied in a shuffled order, unconditionally, so a
    later store can overwrite a smaller value stored by an earlier one.
    Returns (labels, sweeps, invariant_ok) where invariant_ok records that
    L[x] <= x held after every group; with record set, a fourth item lists
    the array after each sweep.
    """
    rng = random.Random(seed)
    src = [int(a) for a in src]
    dst = [int(b) for b in dst]
    L = list(range(n))
    ok = True
    m = len(src)
    states = []
    for s in range(max_sweeps):
        active = False
        for g0 in range(0, m, group):
            stores = []
            for e in range(g0, min(m, g0 + group)):
                targets, values, z = mm_edge_reads(L, src[e], dst[e], order)
                for x, val in zip(targets, values):
                    if val > z:
                        stores.append((x, z))
                        active = True
            rng.shuffle(stores)
            for x, z in stores:
                L[x] = z
            if any(L[x] > x for x in range(n)):
                ok = False
        if record:
            states.append(np.asarray(L, np.int32))
        if not active:
            if record:
                return np.asarray(L, np.int32), s + 1, ok, states
            return np.asarray(L, np.int32), s + 1, ok
    raise RuntimeError("no convergence within %d sweeps" % max_sweeps)


# ------------------------------------------------- sharded (design model) --

def contour_sync_from(src, dst, L0, order: int = 2, max_iter: int = 1 << 20):
    """Algorithm 1's loop (C-Syn, MM^order) started from the labels L0 instead
    of L[i] = i.  L0 must hold L0[x] <= x with L0[x] in x's component of the
    graph the labels belong to.  Returns (labels, iterations)."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    L = np.asarray(L0, np.int64).copy()
    for it in range(1, max_iter + 1):
        Lu = sync_iteration(L, src, dst, order)
        if np.array_equal(Lu, L):
            return L.astype(np.int32), it
        L = Lu
    raise RuntimeError("no convergence within %d iterations" % max_iter)


def sharded_rounds(src, dst, n: int, share, p: int, order: int = 2, max_rounds: int = 1 << 10,
                   record: bool = False):
    """The multi-GPU design on one host: edge e belongs to share share[e] in
    [0, p); every round solves each share from the current labels
    (contour_sync_from) and takes the elementwise minimum of the p results.
    A round that changes nothing ends the run: the labels are then a fixed
    point of MM on every share, hence on the whole edge list.  Returns
    (labels, rounds, states) with states the labels after each round when
    record is set."""
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    share = np.asarray(share)
    L = np.arange(n, dtype=np.int64)
    states = []
    for r in range(1, max_rounds + 1):
        parts = [contour_sync_from(src[share == i], dst[share == i], L, order)[0] for i in range(p)]
        Ln = np.minimum.reduce([q.astype(np.int64) for q in parts]) if parts else L.copy()
        if record:
            states.append(Ln.astype(np.int32))
        if np.array_equal(Ln, L):
            return L.astype(np.int32), r, states
        L = Ln
    raise RuntimeError("no convergence within %d rounds" % max_rounds)


# ------------------------------------------------- incremental (new edges) --

def flatten(L) -> np.ndarray:
    """Every label replaced by the root of its chain (L[x], L[L[x]], ... until
    a fixed point); chains strictly decrease, so this ends."""
    L = np.asarray(L, np.int64).copy()
    while True:
        Ln = L[L]
        if np.array_equal(Ln, L):
            return L.astype(np.int32)
        L = Ln


def add_edges(labels, src, dst, order: int = 2) -> np.ndarray:
    """Labels of G plus the edges (src, dst), given `labels` = the exact
    labels of G (every vertex points at its component's minimum, the old
    root).  The sweeps run, from the old labels (Algorithm 1's loop with a
    warm start), over the new edges plus a tie (x, old root of x) for each
    endpoint x of a new edge; every label is then replaced by the root of its
    chain.  The ties keep an endpoint connected to its old component after
    its own label has been lowered: without them the old edges that made it
    part of that component would have to be swept again."""
    labels = np.asarray(labels, np.int64)
    src = np.asarray(src, np.int64)
    dst = np.asarray(dst, np.int64)
    s = np.concatenate([src, src, dst])
    d = np.concatenate([dst, labels[src], labels[dst]])
    L, _ = contour_sync_from(s, d, labels, order)
    return flatten(L)
