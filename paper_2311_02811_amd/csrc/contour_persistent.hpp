// contour_persistent.hpp -- the on-device sweep loop of one graph, shared by
// the single-graph persistent kernel and the batched multi-workgroup kernel.
#pragma once

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
// Thread 0 only: take the next task of the graph and decide whether the
// workgroup works on it.  Writes the decision to *go and the task to *task.
__device__ __forceinline__ void persistent_next(const SolveArgs& a, int* go_out, long long* task_out)
{
    Ctl* c = a.ctl;
    int go = 0;
    long long t = 0;
    if (__hip_atomic_load(&c->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ST_RUNNING) {
        t = (long long)__hip_atomic_fetch_add(&c->next_task, 1ULL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const long long sweep = t / a.tasks;
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
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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

// Thread 0 only: publish the end of a task (release).
__device__ __forceinline__ void persistent_done(const SolveArgs& a, long long sweep, int any, int anyerr)
{
    Ctl* c = a.ctl;
    if (any)
        __hip_atomic_fetch_max(&c->last_change, (int)sweep + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (anyerr) __hip_atomic_store(&c->range_err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&c->done_task, 1ULL, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// The loop keeps every thread-0 section inside one if-region at the end of
// the body (plus one before the loop), so all lanes of every wave pass the
// same barriers in the same order.
template <int EPT, int BLOCK, bool ATOMIC>
__device__ __forceinline__ void persistent_solve(const SolveArgs& a)
{
    __shared__ long long s_task;
    __shared__ int s_go;
    if (threadIdx.x == 0) persistent_next(a, &s_go, &s_task);
    __syncthreads();
    for (;;) {
        if (!uniform(s_go)) break;
        const long long t = uniform(s_task);
        const long long sweep = t / a.tasks;
        const long long chunk = t - sweep * a.tasks;
        const int order = order_of_sweep(a.sched, (int)sweep);
        int rerr = 0;
        const bool pred = run_tiles_order<EPT, BLOCK, ATOMIC>(a.src, a.dst, a.L, a.L, chunk * a.tiles_per_task,
                                                              a.tiles_per_task, 1, a.m, a.n, order, rerr);
        drain_stores();
        const int any = __syncthreads_or(pred ? 1 : 0);
        const int anyerr = __syncthreads_or(rerr);
        if (threadIdx.x == 0) {
            persistent_done(a, sweep, any, anyerr);
            persistent_next(a, &s_go, &s_task);
        }
        __syncthreads();
    }
}

}  // namespace contour
