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
    long long sweep;         // sweep of the last task taken (-1: none yet)
    int pending;             // tasks of that sweep completed but not yet published
    int changed;             // some published-later task changed a label
    int err;                 // some task met an out-of-range id
    unsigned long long t0;   // the solve's start on the wall clock (Ctl::t0)
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

// Thread 0 only: take the next task of the graph (-1 once the solve has
// ended).  Tasks are taken from the graph's counter in groups of a.take
// consecutive tasks (the host sets a group to about one workgroup's share of
// a sweep), so a workgroup pays the latency of one device-wide atomic per
// group rather than per task; [*grp, *grp_end) is what remains of the
// workgroup's current group.
__device__ __forceinline__ long long persistent_take(const SolveArgs& a, long long* grp, long long* grp_end)
{
    Ctl* c = a.ctl;
    // the rest of a group needs no memory access; the solve's state is read
    // when a new group is taken and whenever a task starts a new sweep
    if (*grp < *grp_end) return (*grp)++;
    if (__hip_atomic_load(&c->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ST_RUNNING) return -1;
    const long long k = a.take > 1 ? a.take : 1;
    const long long t =
        (long long)__hip_atomic_fetch_add(&c->next_task, (unsigned long long)k, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    *grp = t + 1;
    *grp_end = t + k;
    return t;
}

// XCD queues (a.xq_units = U > 0).  The tasks of a sweep are cut into eight
// segments of consecutive tasks, one per XCD (segment x: tasks
// [x T / 8, (x + 1) T / 8) of the T tasks); with edges grouped by destination
// range, a segment covers a few ranges, so the label gathers of an XCD stay
// in its own L2.  Each segment is handed out as U units per sweep; unit j
// holds the tasks j, j + U, j + 2U, ... of the segment, so the U workgroups of
// an XCD (one unit each) walk through the segment side by side, one
// destination range at a time.  Ctl::xq[x] counts the units taken from
// segment x over all sweeps (unit u: sweep u / U, index u % U).  A workgroup
// takes its next unit from its own XCD's queue with one add; before using a
// unit of sweep s it takes, one at a time with a compare-and-swap, any unit
// of an earlier sweep still left in another queue.  So a workgroup starts a
// unit of sweep s only when every unit of every earlier sweep has been taken
// by a running workgroup, and like the single counter the scheme needs no
// co-residency.  Thread 0 only.
struct XcdState {
    int xcd;                  // this workgroup's XCD
    int have;                 // a unit is being worked through
    int q;                    // its queue
    long long sweep;          // its sweep
    long long next_chunk;     // its next task (chunk of the sweep)
    long long end_chunk;      // end of its segment
    long long own_next;       // a unit taken from the own queue and not yet used (-1: none)
};

__device__ __forceinline__ void xcd_segment(const SolveArgs& a, int x, long long* lo, long long* hi)
{
    *lo = (long long)x * a.tasks / 8;
    *hi = (long long)(x + 1) * a.tasks / 8;
}

__device__ __forceinline__ void xcd_use(const SolveArgs& a, XcdState& s, int q, unsigned long long u)
{
    long long lo, hi;
    xcd_segment(a, q, &lo, &hi);
    s.have = 1;
    s.q = q;
    s.sweep = (long long)(u / (unsigned long long)a.xq_units);
    s.next_chunk = lo + (long long)(u % (unsigned long long)a.xq_units);
    s.end_chunk = hi;
}

__device__ __forceinline__ long long persistent_take_xcd(const SolveArgs& a, XcdState& s)
{
    Ctl* c = a.ctl;
    const unsigned long long U = (unsigned long long)a.xq_units;
    for (;;) {
        if (s.have) {
            if (s.next_chunk < s.end_chunk) {
                const long long t = s.sweep * a.tasks + s.next_chunk;
                s.next_chunk += a.xq_units;
                return t;
            }
            s.have = 0;
        }
        if (__hip_atomic_load(&c->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ST_RUNNING) return -1;
        if (s.own_next < 0)
            s.own_next = (long long)__hip_atomic_fetch_add(&c->xq[s.xcd], 1ULL, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long own_sweep = (unsigned long long)s.own_next / U;
        bool stolen = false;
        for (;;) {
            // the untaken unit of the earliest sweep in the other queues,
            // if it is earlier than the own unit
            int best = -1;
            unsigned long long bv = 0;
            for (int d = 1; d < 8; ++d) {
                const int y = (s.xcd + d) & 7;
                const unsigned long long v =
                    __hip_atomic_load(&c->xq[y], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (v / U < own_sweep && (best < 0 || v / U < bv / U)) {
                    best = y;
                    bv = v;
                }
            }
            if (best < 0) break;
            if (__hip_atomic_compare_exchange_strong(&c->xq[best], &bv, bv + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
                xcd_use(a, s, best, bv);
                stolen = true;
                break;
            }
        }
        if (!stolen) {
            xcd_use(a, s, s.xcd, (unsigned long long)s.own_next);
            s.own_next = -1;
        }
    }
}

// XCD of the calling workgroup: workgroups of a launch are dealt to the
// eight XCDs in turn.
__device__ __forceinline__ int xcd_of_workgroup() { return (int)(blockIdx.x & 7); }

// Thread 0 only: start task t (t < 0: the workgroup leaves) and decide
// whether the workgroup works on it.  A task of a later sweep than the last
// one first publishes the workgroup's completed tasks and then waits until
// the previous sweep is complete.
__device__ __forceinline__ int persistent_begin(const SolveArgs& a, PersistentState& w, long long t)
{
    Ctl* c = a.ctl;
    if (t < 0) return 0;
    const long long sweep = t / a.tasks;
    // Another task of the sweep already begun: the sweep was found running
    // then, and neither convergence nor the sweep limit is decided before
    // the sweep is complete, which needs this task too; only the watchdog
    // (a clock read) is checked.  A time-out set meanwhile by a workgroup
    // that waits for this sweep is seen at the next sweep change.
    if (sweep == w.sweep) {
        if (a.watchdog == 0 || wall_clock64() - w.t0 <= a.watchdog) return 1;
        int expect = ST_RUNNING;
        __hip_atomic_compare_exchange_strong(&c->state, &expect, (int)ST_TIMEOUT, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        return 0;
    }
    int go = 0;
    {
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
    return go;
}

// Task `chunk` of a sweep covers tiles [first, first + count): the sweep's
// tiles split evenly over the tasks (sizes differ by at most one tile), and
// the host makes the number of tasks a multiple of the resident workgroups,
// so the workgroups finish a sweep together.
__device__ __forceinline__ void task_tiles(const SolveArgs& a, long long chunk, long long* first, long long* count)
{
    const long long f = chunk * a.ntiles / a.tasks;
    *first = f;
    *count = (chunk + 1) * a.ntiles / a.tasks - f;
}

// Stage cnt labels from global memory g into LDS w, each tagged with
// kLabelClean (see WindowLabels).  Every thread keeps
// kStageUnroll loads in flight before it writes any of them to LDS, 16 bytes
// each when g is 16-byte aligned, so one workgroup has up to 64 KiB of label
// reads outstanding instead of one 4-byte read per thread at a time.  Loads
// and LDS writes are unconditional (indices past the end are clamped to the
// last element, which then receives its own value several times) so that the
// compiler cannot sink a load into a branch and wait for it there.
constexpr int kStageUnroll = 4;

template <int BLOCK>
__device__ __forceinline__ void stage_window(int* w, const int* g, unsigned cnt)
{
    unsigned done = 0;
    if ((reinterpret_cast<uintptr_t>(g) & 15) == 0 && cnt >= 4) {
        const unsigned q = cnt >> 2;
        const int4* g4 = reinterpret_cast<const int4*>(g);
        int4* w4 = reinterpret_cast<int4*>(w);
        for (unsigned i0 = threadIdx.x; i0 < q; i0 += BLOCK * kStageUnroll) {
            int4 v[kStageUnroll];
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u) v[u] = g4[min(i0 + u * BLOCK, q - 1)];
#pragma unroll
            for (int u = 0; u < kStageUnroll; ++u) {
                int4 t = v[u];
                t.x |= kLabelClean;
                t.y |= kLabelClean;
                t.z |= kLabelClean;
                t.w |= kLabelClean;
                w4[min(i0 + u * BLOCK, q - 1)] = t;
            }
        }
        done = q << 2;
    }
    for (unsigned i0 = done + threadIdx.x; i0 < cnt; i0 += BLOCK * kStageUnroll) {
        int v[kStageUnroll];
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u) v[u] = g[min(i0 + u * BLOCK, cnt - 1)];
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u) w[min(i0 + u * BLOCK, cnt - 1)] = v[u] | kLabelClean;
    }
}

// Write the labels of window w that a store lowered (untagged ones) back to
// global memory (g = labels + lo, buffer resource rsrc over the labels, byte
// offset of g in it goff).  Plain mode writes through to memory (sc1 stores: 16 bytes for
// four lowered labels in a row, else 4 bytes each), atomic mode takes the
// atomic minimum of every lowered label (see persistent_solve).  Each thread
// handles four consecutive labels per step (one 16-byte LDS read; the
// window's LDS holds a multiple of 32 labels, so the read stays inside it)
// and kStageUnroll steps at a time.
constexpr int kStoreWriteThrough = 16;  // buffer cache policy: sc1

template <int BLOCK, bool ATOMIC>
__device__ __forceinline__ void write_back_window(const int* w, int* g, __amdgpu_buffer_rsrc_t rsrc,
                                                  unsigned goff, unsigned cnt)
{
    typedef int v4i __attribute__((ext_vector_type(4)));
    const unsigned q = (cnt + 3) >> 2;
    const int4* w4 = reinterpret_cast<const int4*>(w);
    for (unsigned i0 = threadIdx.x; i0 < q; i0 += BLOCK * kStageUnroll) {
        unsigned bits[kStageUnroll];
        int4 val[kStageUnroll];
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u) {
            const unsigned idx = min(i0 + u * BLOCK, q - 1);
            val[u] = w4[idx];
            // lowered labels lack the tag; the lanes of a last, partial
            // quad past cnt hold whatever the LDS held and are masked off
            const unsigned j = idx * 4;
            unsigned b = (val[u].x & kLabelClean ? 0u : 1u) | (val[u].y & kLabelClean ? 0u : 2u) |
                         (val[u].z & kLabelClean ? 0u : 4u) | (val[u].w & kLabelClean ? 0u : 8u);
            if (j + 4 > cnt) b &= (1u << (cnt - j)) - 1u;
            bits[u] = i0 + u * BLOCK < q ? b : 0u;
        }
#pragma unroll
        for (int u = 0; u < kStageUnroll; ++u) {
            const unsigned j = (i0 + u * BLOCK) * 4;
            if (ATOMIC) {
                if (bits[u] & 1u) put<true>(g, (int)j, val[u].x);
                if (bits[u] & 2u) put<true>(g, (int)j + 1, val[u].y);
                if (bits[u] & 4u) put<true>(g, (int)j + 2, val[u].z);
                if (bits[u] & 8u) put<true>(g, (int)j + 3, val[u].w);
            } else if (bits[u] == 15u) {
                const v4i v = {val[u].x, val[u].y, val[u].z, val[u].w};
                __builtin_amdgcn_raw_buffer_store_b128(v, rsrc, goff + j * 4, 0, kStoreWriteThrough);
            } else {
                if (bits[u] & 1u) __builtin_amdgcn_raw_buffer_store_b32(val[u].x, rsrc, goff + j * 4, 0, kStoreWriteThrough);
                if (bits[u] & 2u) __builtin_amdgcn_raw_buffer_store_b32(val[u].y, rsrc, goff + j * 4 + 4, 0, kStoreWriteThrough);
                if (bits[u] & 4u) __builtin_amdgcn_raw_buffer_store_b32(val[u].z, rsrc, goff + j * 4 + 8, 0, kStoreWriteThrough);
                if (bits[u] & 8u) __builtin_amdgcn_raw_buffer_store_b32(val[u].w, rsrc, goff + j * 4 + 12, 0, kStoreWriteThrough);
            }
        }
    }
}

// Windowed task (edges grouped by source block): stage the labels of the
// task's source blocks, plus a margin, in LDS; gather and store there for
// ids inside the window and in global memory otherwise; write the labels the
// task lowered back to global memory once at the end.  Stores into global
// memory follow the write mode (plain or atomic minimum); values staged in
// LDS were read during the sweep, so every label written back is smaller
// than a value the location held during the sweep, exactly as for a direct
// store.
template <int EPT, int BLOCK, bool ATOMIC>
__device__ __forceinline__ bool window_task(const SolveArgs& a, long long first_tile, long long count, int order,
                                            int& rerr, int* nread = nullptr)
{
    extern __shared__ __align__(16) int dyn_lds[];
    __shared__ unsigned s_lo, s_cnt;
    const long long tile_edges = (long long)BLOCK * EPT;
    if (threadIdx.x == 0) {
        const long long e0 = first_tile * tile_edges;
        const long long e1 = std::min(a.m, e0 + count * tile_edges) - 1;
        const unsigned f = (unsigned)a.src[e0], l = (unsigned)a.src[e1];
        // lo rounded down to a multiple of 4 so that the window is staged
        // with 16-byte loads
        const unsigned lo = f < a.n ? ((f >> a.win_shift) << a.win_shift) & ~3u : 0u;
        unsigned long long hi = l < a.n ? ((unsigned long long)((l >> a.win_shift) + 1) << a.win_shift) : a.n;
        hi = std::min<unsigned long long>(a.n, hi + (unsigned)a.win_margin);
        s_lo = lo;
        s_cnt = (unsigned)std::min<unsigned long long>(hi > lo ? hi - lo : 0ULL, (unsigned)a.win_cap);
    }
    __syncthreads();
    const unsigned lo = uniform((int)s_lo);
    const unsigned cnt = uniform((int)s_cnt);
    int* wl = dyn_lds;
    int* hkey = dyn_lds + a.win_cap;
    int* hval = hkey + kHubSlots;
    stage_window<BLOCK>(wl, a.L + lo, cnt);
    for (unsigned i = threadIdx.x; i < (unsigned)kHubSlots; i += BLOCK) {
        hkey[i] = -1;
        hval[i] = 0x7fffffff;
    }
    __syncthreads();
    const WindowLabels lab{wl, lo, cnt, a.L, label_buffer(a.L, a.n), a.n * 4u, hkey, hval};
    const bool pred = run_tiles_lab<EPT, BLOCK, ATOMIC, WindowLabels, 1>(
        a.src, a.dst, lab, first_tile, count, 1, a.m, a.n, order, rerr, nread);
    __syncthreads();
    for (unsigned i = threadIdx.x; i < (unsigned)kHubSlots; i += BLOCK) {
        const int k = hkey[i];
        if (k >= 0) __hip_atomic_fetch_min(a.L + k, hval[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    write_back_window<BLOCK, ATOMIC>(wl, a.L + lo, lab.rsrc, lo * 4u, cnt);
    return pred;
}

// Label stores into global memory are coherent across the XCDs in every
// write mode: atomic minima, or (window write-back in plain mode) stores
// written through to memory.  The early convergence check needs every read
// of the last sweep to see the labels' final values.  With ordinary cached
// stores, workgroups on different XCDs racing on one cache line (the lost
// updates of the asynchronous update) could leave an XCD holding, in its own
// L2, a line it wrote itself with a smaller label than memory ended up with;
// the sweep-boundary release/acquire (agent or system scope) did not refresh
// it, and a sweep then passed as unchanged over an edge whose endpoints
// differ (observed on the MI355X in batched solves: a few vertices of 1 to 3
// of 916 graphs, in some launches; none with the coherent stores).  Stores
// into a label window in LDS, which one workgroup owns, follow the write
// mode (plain or atomic minimum).
//
// The task loop.  Its thread-0 sections (take a task; begin it, which may
// spin) each end at a barrier, and all loop control is read back from LDS
// through readfirstlane, so every lane of a wave passes the same barriers in
// the same order.  The convergence decision reads last_change only after
// done_task shows every task of the previous sweep published, and each
// publication adds to done_task with release semantics after its
// last_change update, so a sweep that changed a label is never mistaken for
// one that did not.
template <int EPT, int BLOCK, bool ATOMIC, bool WIN = false, bool XQ = false>
__device__ __forceinline__ void persistent_solve(const SolveArgs& a)
{
    // s_task is read by every wave at the top of an iteration and rewritten
    // by thread 0 only after the next barrier; the next task goes through
    // s_next, because without a barrier inside a task (no label window) a
    // fast wave 0 would otherwise overwrite s_task before a slow wave has
    // read it, and that wave would work on the wrong task.
    __shared__ long long s_task, s_next;
    __shared__ int s_go;
    PersistentState w{-1, 0, 0, 0, 0};
    long long grp = 0, grp_end = 0;  // thread 0: the rest of its task group
    // thread 0's XCD-queue state lives in LDS: kept in registers across the
    // task loop it would push the tile code into spilling
    __shared__ XcdState xs;
    if (XQ && threadIdx.x == 0) xs = XcdState{xcd_of_workgroup(), 0, 0, 0, 0, 0, -1};
    if (threadIdx.x == 0) {
        w.t0 = a.ctl->t0;
        const long long t = XQ ? persistent_take_xcd(a, xs) : persistent_take(a, &grp, &grp_end);
        s_go = persistent_begin(a, w, t);
        s_task = t;
    }
    __syncthreads();
    // per thread: some task since the last publication changed a label /
    // met an out-of-range id
    int changed = 0, rerr = 0;
    int nread = 0;  // instrumented solve: label reads of this thread
    int* const count_reads = a.reads ? &nread : nullptr;
    for (;;) {
        if (!uniform(s_go)) break;
        const long long t = uniform(s_task);
        const long long sweep = t / a.tasks;
        long long first, count;
        task_tiles(a, t - sweep * a.tasks, &first, &count);
        const int order = order_of_sweep(a.sched, (int)sweep);
        bool pred;
        if (WIN)
            pred = window_task<EPT, BLOCK, ATOMIC>(a, first, count, order, rerr, count_reads);
        else
            pred = run_tiles_order<EPT, BLOCK, true>(a.src, a.dst, a.L, a.L, first, count, 1, a.m, a.n, order,
                                                     rerr, count_reads);
        changed |= pred ? 1 : 0;
        // take the next task; only a move to another sweep (or the end)
        // publishes, which needs every store of the workgroup drained and
        // the per-thread flags combined
        if (threadIdx.x == 0) s_next = XQ ? persistent_take_xcd(a, xs) : persistent_take(a, &grp, &grp_end);
        __syncthreads();
        const long long next = uniform(s_next);
        const bool leave = next < 0 || next / a.tasks != sweep;
        int any = 0, anyerr = 0;
        if (leave) {
            drain_stores();
            any = __syncthreads_or(changed);
            anyerr = __syncthreads_or(rerr);
            changed = 0;
            rerr = 0;
        }
        if (threadIdx.x == 0) {
            w.pending += 1;
            w.changed |= any;
            w.err |= anyerr;
            s_go = persistent_begin(a, w, next);
            s_task = next;
        }
        __syncthreads();
    }
    if (a.reads) {
        // instrumented solve: one global add per workgroup
        __shared__ unsigned long long s_reads;
        if (threadIdx.x == 0) s_reads = 0;
        __syncthreads();
        atomicAdd(&s_reads, (unsigned long long)nread);
        __syncthreads();
        if (threadIdx.x == 0) atomicAdd(a.reads, s_reads);
    }
}

}  // namespace contour
