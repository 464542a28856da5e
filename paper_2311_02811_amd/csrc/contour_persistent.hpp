// contour_persistent.hpp -- the on-device sweep loop of one graph, shared by
// the single-graph persistent kernel and the batched multi-workgroup kernel.
#pragma once

#include <algorithm>

#include "contour_device.hpp"

namespace contour {

// Work on one graph until its solve ends.  Task t covers edge chunk t % T of
// sweep t / T (T tasks per sweep).  A workgroup takes the next task from the
// graph's counter; before working on sweep s it waits until all T tasks of
// sweep s-1 are done, and if sweep s-1 changed nothing the solve has
// converged.  A workgroup only ever waits for tasks that running workgroups
// have already taken, so the scheme needs no co-residency and cannot
// deadlock.  Task completion is a release (label stores drained, then an
// agent-scope release add) and the wait ends with an acquire, so sweep s
// reads every store of sweeps < s.  Returns when the graph's solve has ended
// (converged, sweep limit or watchdog); several workgroups may return for
// the same graph.
// Per-workgroup bookkeeping of the persistent loop (thread 0 only).
// Completed tasks are published once per sweep: when the workgroup moves on
// to a later sweep it first releases its stores (agent-scope release) and
// adds its count to done_task, and only then may it wait for that sweep to
// be complete.  A workgroup therefore issues one release, one done_task
// add and one acquire per sweep it takes part in, instead of one per task.
struct PersistentState {
    long long sweep;    // sweep of the last task taken (-1: none yet)
    int pending;        // tasks of that sweep completed but not yet published
    int changed;        // some published-later task changed a label
    int err;            // some task met an out-of-range id
};

__device__ __forceinline__ void persistent_publish(const SolveArgs& a, PersistentState& w)
{
    if (w.pending == 0) return;
    Ctl* c = a.ctl;
    if (w.changed)
        __hip_atomic_fetch_max(&c->last_change, (int)w.sweep + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (w.err) __hip_atomic_store(&c->range_err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&c->done_task, (unsigned long long)w.pending, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    w.pending = 0;
    w.changed = 0;
    w.err = 0;
}

// Thread 0 only: take the next task of the graph and decide whether the
// workgroup works on it.
__device__ __forceinline__ void persistent_next(const SolveArgs& a, PersistentState& w, int* go_out,
                                                long long* task_out)
{
    Ctl* c = a.ctl;
    int go = 0;
    long long t = 0;
    if (__hip_atomic_load(&c->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ST_RUNNING) {
        t = (long long)__hip_atomic_fetch_add(&c->next_task, 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const long long sweep = t / a.tasks;
        if (sweep != w.sweep) {
            // leaving w.sweep for good: publish it before waiting on sweep - 1
            persistent_publish(a, w);
            if (sweep > 0) {
                const unsigned long long need = (unsigned long long)(sweep * a.tasks);
                while (__hip_atomic_load(&c->done_task, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    if (__hip_atomic_load(&c->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ST_RUNNING)
                        break;
                    if (watchdog_expired(c, a.watchdog)) {
                        int expect = ST_RUNNING;
                        __hip_atomic_compare_exchange_strong(&c->state, &expect, (int)ST_TIMEOUT, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            w.sweep = sweep;
        }
        if (__hip_atomic_load(&c->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ST_RUNNING) {
            const int lc = __hip_atomic_load(&c->last_change, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int st = ST_RUNNING;
            if (sweep > 0 && lc <= sweep - 1)
                st = ST_CONVERGED;
            else if (a.max_sweeps > 0 && sweep >= a.max_sweeps)
                st = ST_LIMIT;
            else if (watchdog_expired(c, a.watchdog))
                st = ST_TIMEOUT;
            if (st == ST_RUNNING) {
                go = 1;
            } else {
                int expect = ST_RUNNING;
                if (__hip_atomic_compare_exchange_strong(&c->state, &expect, st, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT))
                    __hip_atomic_store(&c->sweeps, (int)sweep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    *go_out = go;
    *task_out = t;
}

// The loop keeps every thread-0 section inside one if-region at the end of
// the body (plus one before the loop), so all lanes of every wave pass the
// same barriers in the same order.  The convergence decision reads
// last_change only after done_task shows every task of the previous sweep
// published, and each publication adds to done_task with release semantics
// after its last_change update, so a sweep that changed a label is never
// mistaken for one that did not.
// Windowed task (edges grouped by source block): stage the labels of the
// task's source blocks, plus a margin, in LDS; gather and store there for
// ids inside the window and in global memory otherwise; write the labels the
// task lowered back to global memory once at the end.  Stores into global
// memory follow the write mode (plain or atomic minimum); values staged in
// LDS were read during the sweep, so every label written back is smaller
// than a value the location held during the sweep, exactly as for a direct
// store.
template <int EPT, int BLOCK, bool ATOMIC>
__device__ __forceinline__ bool window_task(const SolveArgs& a, long long first_tile, int order, int& rerr)
{
    extern __shared__ int dyn_lds[];
    __shared__ unsigned s_lo, s_cnt;
    const long long tile_edges = (long long)BLOCK * EPT;
    if (threadIdx.x == 0) {
        const long long e0 = first_tile * tile_edges;
        const long long e1 = std::min(a.m, e0 + (long long)a.tiles_per_task * tile_edges) - 1;
        const unsigned f = (unsigned)a.src[e0], l = (unsigned)a.src[e1];
        const unsigned lo = f < a.n ? (f >> a.win_shift) << a.win_shift : 0u;
        unsigned long long hi = l < a.n ? ((unsigned long long)((l >> a.win_shift) + 1) << a.win_shift) : a.n;
        hi = std::min<unsigned long long>(a.n, hi + (unsigned)a.win_margin);
        s_lo = lo;
        s_cnt = (unsigned)std::min<unsigned long long>(hi > lo ? hi - lo : 0ULL, (unsigned)a.win_cap);
    }
    __syncthreads();
    const unsigned lo = uniform((int)s_lo);
    const unsigned cnt = uniform((int)s_cnt);
    int* wl = dyn_lds;
    unsigned* dirty = reinterpret_cast<unsigned*>(dyn_lds + a.win_cap);
    for (unsigned i = threadIdx.x; i < cnt; i += BLOCK) wl[i] = a.L[lo + i];
    for (unsigned i = threadIdx.x; i < (cnt + 31) / 32; i += BLOCK) dirty[i] = 0;
    __syncthreads();
    const WindowLabels lab{wl, dirty, lo, cnt, a.L};
    const bool pred = run_tiles_lab<EPT, BLOCK, ATOMIC, WindowLabels, (EPT <= 2 ? 4 : 2)>(
        a.src, a.dst, lab, first_tile, a.tiles_per_task, 1, a.m, a.n, order, rerr);
    __syncthreads();
    for (unsigned i = threadIdx.x; i < cnt; i += BLOCK)
        if ((dirty[i >> 5] >> (i & 31)) & 1u) put<ATOMIC>(a.L, (int)(lo + i), wl[i]);
    return pred;
}

template <int EPT, int BLOCK, bool ATOMIC, bool WIN = false>
__device__ __forceinline__ void persistent_solve(const SolveArgs& a)
{
    __shared__ long long s_task;
    __shared__ int s_go;
    PersistentState w{-1, 0, 0, 0};
    if (threadIdx.x == 0) persistent_next(a, w, &s_go, &s_task);
    __syncthreads();
    for (;;) {
        if (!uniform(s_go)) break;
        const long long t = uniform(s_task);
        const long long sweep = t / a.tasks;
        const long long chunk = t - sweep * a.tasks;
        const int order = order_of_sweep(a.sched, (int)sweep);
        int rerr = 0;
        bool pred;
        if (WIN)
            pred = window_task<EPT, BLOCK, ATOMIC>(a, chunk * a.tiles_per_task, order, rerr);
        else
            pred = run_tiles_order<EPT, BLOCK, ATOMIC>(a.src, a.dst, a.L, a.L, chunk * a.tiles_per_task,
                                                       a.tiles_per_task, 1, a.m, a.n, order, rerr);
        drain_stores();
        const int any = __syncthreads_or(pred ? 1 : 0);
        const int anyerr = __syncthreads_or(rerr);
        if (threadIdx.x == 0) {
            w.pending += 1;
            w.changed |= any;
            w.err |= anyerr;
            persistent_next(a, w, &s_go, &s_task);
        }
        __syncthreads();
    }
}

}  // namespace contour
