// contour_single.hip -- single-graph solve: label initialisation, the sweep
// drivers (persistent on-device sequencing and host-sequenced sweeps), the
// synchronous C-Syn variant, and the contour_cc / contour_cc_ex entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "contour.h"
#include "contour_device.hpp"
#include "contour_persistent.hpp"
#include "contour_runtime.hpp"

namespace contour {

// ------------------------------------------------------------ set-up ----

__global__ void k_reset_ctl(Ctl* c)
{
    int* p = reinterpret_cast<int*>(c);
    if (threadIdx.x < sizeof(Ctl) / sizeof(int)) p[threadIdx.x] = 0;
    __syncthreads();
    if (threadIdx.x == 0) c->t0 = wall_clock64();
}

// Algorithm 1, initialisation: L[i] = i.  For a warm start, check instead that
// every label satisfies 0 <= L[i] <= i, which keeps every chain the sweeps
// follow inside [0, n); a violation stops the solve before any sweep.
__global__ void k_init_labels(int* L, unsigned n, int warm, Ctl* c)
{
    bool bad = false;
    for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (!warm)
            L[i] = (int)i;
        else {
            int x = L[i];
            bad |= x < 0 || (unsigned)x > i;
        }
    }
    if (bad) __hip_atomic_store(&c->state, (int)ST_BAD_START, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_write_stats(const Ctl* c, contour_stats_t* out, int range_err)
{
    if (threadIdx.x != 0) return;
    int status = CONTOUR_OK;
    if (c->state == ST_BAD_START)
        status = CONTOUR_EINVAL;
    else if (c->range_err || range_err)
        status = CONTOUR_ERANGE;
    else if (c->state == ST_LIMIT || c->state == ST_TIMEOUT)
        status = CONTOUR_ENOCONV;
    out->status = status;
    out->sweeps_executed = c->sweeps;
    out->sweeps_with_writes = c->last_change;
    out->reserved = 0;
}

// ------------------------------------------------- persistent driver ----
// One launch for the whole solve; the sweep loop is persistent_solve() in
// contour_persistent.hpp.
template <int EPT, int BLOCK, bool ATOMIC, bool WIN, bool XQ = false>
__global__ __launch_bounds__(BLOCK) void k_persistent(SolveArgs a)
{
    persistent_solve<EPT, BLOCK, ATOMIC, WIN, XQ>(a);
}

// ------------------------------------------------- host-loop driver -----
// One launch per sweep; kernel boundaries order the sweeps.  Sweep s first
// looks at what sweep s-1 recorded: if it changed nothing (or the sweep limit
// is reached, or the solve already ended) the kernel returns at once, so the
// host may enqueue several sweeps ahead and only check every few.
// R is read, W written: the same array for the asynchronous update; for the
// synchronous update (Algorithm 1) W = L_u was filled with a copy of R first.
template <int EPT, int BLOCK, bool ATOMIC>
__global__ __launch_bounds__(BLOCK) void k_sweep(SolveArgs a, const int* R, int* W, int sweep)
{
    Ctl* c = a.ctl;
    if (c->state != ST_RUNNING) return;
    int st = ST_RUNNING;
    if (sweep > 0 && c->last_change <= sweep - 1)
        st = ST_CONVERGED;
    else if (a.max_sweeps > 0 && sweep >= a.max_sweeps)
        st = ST_LIMIT;
    else if (watchdog_expired(c, a.watchdog))
        st = ST_TIMEOUT;
    if (st != ST_RUNNING) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            c->state = st;
            c->sweeps = sweep;
        }
        return;
    }
    const int order = order_of_sweep(a.sched, sweep);
    const long long tile_edges = (long long)BLOCK * EPT;
    const long long ntiles = (a.m + tile_edges - 1) / tile_edges;
    bool pred = false;
    int rerr = 0;
    const long long mine = blockIdx.x < ntiles ? (ntiles - blockIdx.x + gridDim.x - 1) / gridDim.x : 0;
    pred = run_tiles_order<EPT, BLOCK, ATOMIC>(a.src, a.dst, R, W, blockIdx.x, mine, gridDim.x, a.m, a.n,
                                               order, rerr);
    const int any = uniform(__syncthreads_or(pred ? 1 : 0));
    const int anyerr = uniform(__syncthreads_or(rerr));
    if (threadIdx.x == 0) {
        if (any) c->last_change = sweep + 1;
        if (anyerr) c->range_err = 1;
    }
}

// Synchronous update: L_u = L before the sweep (skipped once the solve ended).
__global__ void k_copy_labels(const int* R, int* W, unsigned n, const Ctl* c)
{
    if (c->state != ST_RUNNING) return;
    for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) W[i] = R[i];
}

// Edges added to a labelled graph: edge i of the new list becomes three
// edges of the augmented list, (w, v), (w, L[w]) and (v, L[v]), where L holds
// the graph's exact labels (every vertex points at its component's minimum,
// its old root).  The two ties keep an endpoint joined to its old component
// after the sweeps lower its own label, so the old edges never need another
// sweep.  An id outside [0, n) is copied unchanged (no label read) and the
// sweep's range check reports it.
__global__ void k_tie_edges(const int* __restrict__ src, const int* __restrict__ dst, long long m,
                            const int* __restrict__ L, unsigned n, int* __restrict__ as, int* __restrict__ ad)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m; i += (long long)gridDim.x * blockDim.x) {
        const int w = src[i], v = dst[i];
        as[i] = w;
        ad[i] = v;
        as[m + i] = w;
        ad[m + i] = (unsigned)w < n ? L[w] : w;
        as[2 * m + i] = v;
        ad[2 * m + i] = (unsigned)v < n ? L[v] : v;
    }
}

// Every label replaced by the root of its chain (L[x], L[L[x]], ... until
// L[r] = r).  Chains strictly decrease, so the walk ends; concurrent walks
// only replace a label by another vertex of the same chain.  Skipped when
// the warm start was refused (the labels are then left as they were).
__global__ void k_flatten(int* L, unsigned n, const Ctl* c)
{
    if (c->state == ST_BAD_START) return;
    for (unsigned x = blockIdx.x * blockDim.x + threadIdx.x; x < n; x += gridDim.x * blockDim.x) {
        unsigned r = (unsigned)L[x];
        for (;;) {
            const unsigned q = (unsigned)L[r];
            if (q >= r) break;
            r = q;
        }
        L[x] = (int)r;
    }
}

// ------------------------------------------------ measurement ----------
// Ceiling of a sweep's memory access pattern without its arithmetic: stream
// the edge arrays and (mode 1) gather L[dst], (mode 2) gather L[src] and
// L[dst], summing what was read.  Workgroup b works on segment b & 7 of the
// edge list (workgroups are dealt to the eight XCDs in turn), so on a copy
// grouped by destination range each XCD gathers from its own ranges, as the
// sweep's XCD queues arrange it.  Four edges per thread per step, read with
// one 16-byte load per array when both arrays are 16-byte aligned (segments
// start on multiples of four edges), else one load per edge.
__device__ __forceinline__ int ceiling_gathers(const int* __restrict__ L, unsigned n, int mode, const int (&w)[4],
                                               const int (&v)[4], const bool (&ok)[4])
{
    int acc = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        acc ^= w[k] ^ v[k];
        if (ok[k] && mode >= 1 && (unsigned)v[k] < n) acc += L[v[k]];
        if (ok[k] && mode >= 2 && (unsigned)w[k] < n) acc += L[w[k]];
    }
    return acc;
}

__global__ __launch_bounds__(1024) void k_gather_ceiling(const int* __restrict__ src, const int* __restrict__ dst,
                                                         long long m, const int* __restrict__ L, unsigned n,
                                                         int mode, int* __restrict__ sink)
{
    const int x = blockIdx.x & 7;
    const long long per = gridDim.x / 8, j = blockIdx.x / 8;
    const long long lo = ((long long)x * m / 8) & ~3LL;
    const long long hi = x == 7 ? m : (((long long)x + 1) * m / 8) & ~3LL;
    const bool vec = ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0;
    int acc = 0;
    for (long long e = lo + (j * 1024 + threadIdx.x) * 4; e < hi; e += per * 4096) {
        int w[4], v[4];
        bool ok[4];
        if (vec && e + 4 <= hi) {
            const edge4_t a = __builtin_nontemporal_load(reinterpret_cast<const edge4_t*>(src + e));
            const edge4_t b = __builtin_nontemporal_load(reinterpret_cast<const edge4_t*>(dst + e));
            w[0] = a.x, w[1] = a.y, w[2] = a.z, w[3] = a.w;
            v[0] = b.x, v[1] = b.y, v[2] = b.z, v[3] = b.w;
#pragma unroll
            for (int k = 0; k < 4; ++k) ok[k] = true;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                ok[k] = e + k < hi;
                const long long i = ok[k] ? e + k : hi - 1;
                w[k] = ld_edge(src + i);
                v[k] = ld_edge(dst + i);
            }
        }
        acc += ceiling_gathers(L, n, mode, w, v, ok);
    }
    if (acc == 0x7fffffff) sink[0] = acc;  // keeps the reads; practically never taken
}

// ----------------------------------------------------- dispatch ---------

typedef void (*persistent_fn)(SolveArgs);
typedef void (*sweep_fn)(SolveArgs, const int*, int*, int);

// Register limits: 1024-thread workgroups get at most 128 registers per
// lane and 512-thread ones 256.  Edges per thread of the persistent loop are
// capped where the compiler would otherwise spill: eight become four with
// 1024 threads.
template <int BLOCK, bool WIN>
struct EptCap {
    static constexpr int e8 = BLOCK == 1024 ? 4 : 8;
    static constexpr int e4 = 4;
};

template <int BLOCK, bool ATOMIC, bool WIN>
static void pick(int ept, persistent_fn* p, sweep_fn* s)
{
    constexpr int e4 = EptCap<BLOCK, WIN>::e4;
    constexpr int e8 = EptCap<BLOCK, WIN>::e8 < e4 ? e4 : EptCap<BLOCK, WIN>::e8 == 4 ? e4 : 8;
    switch (ept) {
    // the host-loop sweep stores into global memory with atomic minima in
    // either write mode (see run_hostloop)
    case 1: *p = k_persistent<1, BLOCK, ATOMIC, WIN>; *s = k_sweep<1, BLOCK, true>; break;
    case 2: *p = k_persistent<2, BLOCK, ATOMIC, WIN>; *s = k_sweep<2, BLOCK, true>; break;
    case 4: *p = k_persistent<e4, BLOCK, ATOMIC, WIN>; *s = k_sweep<4, BLOCK, true>; break;
    default: *p = k_persistent<e8, BLOCK, ATOMIC, WIN>; *s = k_sweep<(BLOCK == 1024 ? 4 : 8), BLOCK, true>; break;
    }
}

template <bool WIN>
static void pick_w(int block, int ept, bool atomic, persistent_fn* p, sweep_fn* s)
{
    if (block == 1024) {
        if (atomic) pick<1024, true, WIN>(ept, p, s);
        else pick<1024, false, WIN>(ept, p, s);
    } else if (block == 512) {
        if (atomic) pick<512, true, WIN>(ept, p, s);
        else pick<512, false, WIN>(ept, p, s);
    } else {
        if (atomic) pick<256, true, WIN>(ept, p, s);
        else pick<256, false, WIN>(ept, p, s);
    }
}

static void pick_kernels(int block, int ept, bool atomic, persistent_fn* p, sweep_fn* s, bool win = false)
{
    if (win) pick_w<true>(block, ept, atomic, p, s);
    else pick_w<false>(block, ept, atomic, p, s);
}

// Window kernels with XCD queues (edges grouped by destination range):
// 1024-thread workgroups with 2 or 4 edges per thread; null otherwise.
static persistent_fn pick_xq(int block, int ept, bool atomic)
{
    if (block != 1024) return nullptr;
    if (ept == 2) return atomic ? k_persistent<2, 1024, true, true, true> : k_persistent<2, 1024, false, true, true>;
    if (ept == 4) return atomic ? k_persistent<4, 1024, true, true, true> : k_persistent<4, 1024, false, true, true>;
    return nullptr;
}

// Destination ranges of 2^19 ids: 2 MiB of labels, half an XCD's L2.
constexpr int kDstRangeShift = 19;

int dst_range_shift(const Resolved& r, long long m, int n)
{
    if (r.dst_ranges == CONTOUR_DST_RANGES_OFF || r.driver != CONTOUR_DRIVER_PERSISTENT) return 0;
    if (r.dst_ranges == CONTOUR_DST_RANGES_ON) return kDstRangeShift;
    if (r.dst_ranges >= 16) return r.dst_ranges;  // ranges of 2^dst_ranges ids
    // automatic: where the labels outgrow one XCD's L2 (4 MiB) and the graph
    // has enough edges per vertex to repay the second pass
    return n > (1 << 20) && m >= 4LL * n ? kDstRangeShift : 0;
}

void solve_reorder_geometry(const DeviceInfo& d, const Resolved& r, long long m, int n, Reorder* ro)
{
    reorder_geometry(d, m, n, ro, dst_range_shift(r, m, n));
}

bool wants_reorder(const Resolved& r, long long m, int n)
{
    if (m >= 0x7fffffffLL) return false;  // slots of the counting sort are int32
    if (r.reorder == CONTOUR_REORDER_ON) return true;
    if (r.reorder == CONTOUR_REORDER_OFF) return false;
    return reorder_auto(m, n);
}

// Geometry: 256-thread workgroups; edges per thread grow with m so that small
// graphs still spread over many workgroups and large ones get memory-level
// parallelism; persistent tasks aim at several tasks per workgroup and sweep.
// Geometry.  Large graphs: 1024-thread workgroups (one per CU) with four
// edges per thread.  Small graphs: 256-thread workgroups and one or two
// edges per thread, so that the edges still spread over many workgroups.
static void auto_geometry(const DeviceInfo& d, long long m, Resolved* r)
{
    (void)d;
    const bool large = m >= (4LL << 20);
    if (r->block == 0) r->block = large ? 1024 : 256;
    if (r->ept == 0) r->ept = large ? 4 : (m >= (1LL << 20) ? 2 : 1);
}

// Persistent tasks: every task takes one counter increment, and every
// workgroup publishes once per sweep, so tasks are large: m / 256 edges,
// between 4096 and 65536.  A single graph below 4 M edges takes m / 64 edges
// per task (at least 4096), so its solve runs on about 64 workgroups: each
// works through more consecutive edges per sweep, which carries labels
// further within a sweep (measured on the MI355X: ER with 524,288 edges 2
// sweeps and 0.141 ms against 3 sweeps and 0.164 ms on 128 workgroups; with
// 2 M edges 0.33 ms against 0.39).  Many graphs solved side by side (batched
// plans) keep m / 256.
static int auto_tiles_per_task(long long m, long long tile_edges, bool solo)
{
    long long want = std::max<long long>(4096, std::min<long long>(65536, m / 256));
    if (solo && m < (4LL << 20)) want = std::max<long long>(4096, m / 64);
    return (int)std::max<long long>(1, want / tile_edges);
}

int prepare_persistent(const DeviceInfo& d, const Resolved& r0, const int* src, const int* dst,
                       long long m, int n, int* L, Ctl* ctl, int* ws, PersistentLaunch* out)
{
    Resolved r = r0;
    const bool reorder = m > 0 && wants_reorder(r0, m, n);
    if (reorder) {
        // label windows fill the LDS of a CU: one 1024-thread workgroup each
        if (r.block == 0) r.block = 1024;
        if (r.ept == 0) r.ept = m >= (4LL << 20) ? 4 : 2;
    }
    auto_geometry(d, m, &r);
    PersistentLaunch p;
    p.src_in = src;
    p.dst_in = dst;
    p.reorder = reorder;
    if (p.reorder) {
        if (!ws) return CONTOUR_EINVAL;
        solve_reorder_geometry(d, r0, m, n, &p.ro);
        reorder_bind(&p.ro, ws);
        src = p.ro.src2;
        dst = p.ro.dst2;
    }
    p.n = n;
    p.warm = r.warm ? 1 : 0;
    p.init_blocks = (unsigned)std::max<long long>(
        1, std::min<long long>(((long long)n + 255) / 256, (long long)d.cus * 8));
    p.block = r.block;
    SolveArgs& a = p.args;
    a.src = src;
    a.dst = dst;
    a.L = L;
    a.m = m;
    a.n = (unsigned)n;
    a.sched = r.sched;
    a.max_sweeps = r.max_sweeps;
    a.ctl = ctl;
    a.watchdog = watchdog_ticks(d);
    a.tiles_per_task = 1;
    a.tasks = 0;
    a.ntiles = 0;
    a.take = 1;
    a.win_cap = 0;
    a.win_shift = 0;
    a.win_margin = 0;
    a.xq_units = 0;
    p.kernel = nullptr;
    p.grid = 0;
    p.lds = 0;
    if (m > 0) {
        sweep_fn ks;
        // label windows read global labels through 32-bit buffer offsets
        const bool win = p.reorder && n < (1 << 30);
        pick_kernels(r.block, r.ept, r.atomic, &p.kernel, &ks, win);
        // edges grouped by destination range: the XCD-queue kernel
        persistent_fn kxq = win && p.ro.R > 0 ? pick_xq(r.block, r.ept, r.atomic) : nullptr;
        if (kxq) std::swap(p.kernel, kxq);
        if (win) {
            // the largest window that fits the LDS of one workgroup, a
            // multiple of 32 labels (after the hub table of out-of-window
            // stores)
            const long long bytes = std::max(0, d.max_lds_per_block - 2048 - 8 * kHubSlots);
            long long cap = (bytes / 4) & ~31LL;
            if (r.window > 0) cap = std::min<long long>(cap, (long long)r.window & ~31LL);
            a.win_cap = (int)std::min<long long>(cap, ((long long)n + 31) & ~31LL);
            a.win_shift = p.ro.shift;
            a.win_margin = std::max(1, (1 << p.ro.shift) / 2);
            if (kxq) {
                // a task's window spans exactly its first to last source id:
                // with destination ranges a task holds a few blocks' edges of
                // one range, with no locality for a margin to catch
                a.win_shift = 0;
                a.win_margin = 0;
            }
            p.lds = (size_t)a.win_cap * 4 + (size_t)kHubSlots * 8;
            CONTOUR_HIP(hipFuncSetAttribute((const void*)p.kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)p.lds));
            if (kxq)
                CONTOUR_HIP(hipFuncSetAttribute((const void*)kxq, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                (int)p.lds));
        }
        const long long tile_edges = (long long)r.block * r.ept;
        const long long ntiles = (m + tile_edges - 1) / tile_edges;
        int occ = 0;
        CONTOUR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)p.kernel, r.block, p.lds));
        const long long resident = (long long)std::max(occ, 1) * d.cus;
        int tpt = r.chunk_tiles ? r.chunk_tiles : auto_tiles_per_task(m, tile_edges, r.solo);
        if (win && !r.chunk_tiles) {
            // A window is staged per task.  Tasks of 32 Ki edges, about one
            // source block of a sparse graph; where blocks hold many more
            // edges than that (dense graphs), 16 Ki, so that a block's
            // window is staged afresh, with the other workgroups' updates,
            // several times per sweep (measured: fewer sweeps on R-MAT).
            const long long per_block = m / std::max(1, p.ro.K);
            long long want = per_block > 65536 ? 16384 : 32768;
            if (kxq) {
                // destination ranges: a task of E consecutive edges spans
                // about E n R / m source ids; E is the largest number of
                // whole tiles whose span fits the window (measured on R-MAT
                // scale 24: 16 Ki-edge tasks, 8.9 ms for 4 sweeps, against
                // 9.4 ms with 12 Ki and 10.4 ms with 8 Ki)
                want = (long long)((double)a.win_cap * (double)m / ((double)n * p.ro.R));
            }
            tpt = (int)std::max<long long>(1, want / tile_edges);
        }
        // the sweep's tiles split evenly over a number of tasks that is a
        // multiple of the workgroups, so that they finish a sweep together
        const long long g = r.grid ? r.grid : resident;
        long long tasks = (ntiles + tpt - 1) / tpt;
        if (tasks > g) tasks = std::min<long long>(ntiles, (tasks + g - 1) / g * g);
        a.ntiles = ntiles;
        a.tasks = tasks;
        a.tiles_per_task = (int)((ntiles + tasks - 1) / tasks);
        p.grid = (unsigned)std::min<long long>(g, a.tasks);
        // each workgroup takes its share of a sweep with one atomic
        a.take = (int)std::max<long long>(1, a.tasks / p.grid);
        // edges grouped by destination range: per-XCD queues, one unit per
        // workgroup and sweep (the grid must split evenly over the XCDs)
        if (kxq) {
            if (p.grid % 8 == 0)
                a.xq_units = (int)(p.grid / 8);
            else
                std::swap(p.kernel, kxq);  // back to the single-counter window kernel
        }
    }
    *out = p;
    return CONTOUR_OK;
}

int enqueue_persistent(const PersistentLaunch& p, contour_stats_t* stats, hipStream_t stream,
                       hipEvent_t ev_begin, hipEvent_t ev_end)
{
    Ctl* ctl = p.args.ctl;
    if (p.reorder) {
        int rc = enqueue_reorder(p.ro, p.src_in, p.dst_in, stream);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(64), 0, stream, ctl);
    hipLaunchKernelGGL(k_init_labels, dim3(p.init_blocks), dim3(256), 0, stream, p.args.L,
                       (unsigned)p.n, p.warm, ctl);
    CONTOUR_HIP(hipGetLastError());
    if (ev_begin) CONTOUR_HIP(hipEventRecord(ev_begin, stream));
    if (p.kernel) {
        hipLaunchKernelGGL(p.kernel, dim3(p.grid), dim3(p.block), p.lds, stream, p.args);
        CONTOUR_HIP(hipGetLastError());
    }
    if (ev_end) CONTOUR_HIP(hipEventRecord(ev_end, stream));
    if (stats) {
        hipLaunchKernelGGL(k_write_stats, dim3(1), dim3(64), 0, stream, (const Ctl*)ctl, stats, 0);
        CONTOUR_HIP(hipGetLastError());
    }
    return CONTOUR_OK;
}

int enqueue_empty_stats(Ctl* ctl, contour_stats_t* stats, int range_err, hipStream_t stream)
{
    hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(64), 0, stream, ctl);
    hipLaunchKernelGGL(k_write_stats, dim3(1), dim3(64), 0, stream, (const Ctl*)ctl, stats, range_err);
    CONTOUR_HIP(hipGetLastError());
    return CONTOUR_OK;
}

// Host-sequenced sweeps (asynchronous or synchronous update).  Blocks the
// calling thread: it reads the control block every few sweeps.  Label
// stores are atomic minima in either write mode: with plain global stores
// one R-MAT scale-24 solve in about 25 on the MI355X ended with wrong labels
// (status OK, sweep counts as usual; not seen again in 22 repeats, cause not
// found), so, as inside the persistent kernels, plain stores are kept to
// memory that one workgroup owns (LDS windows, one-workgroup graphs).
static int run_hostloop(const DeviceInfo& d, const Resolved& r0, const int* src, const int* dst,
                        long long m, int n, int* L, Workspace* ws, contour_stats_t* stats,
                        hipStream_t stream)
{
    Resolved r = r0;
    auto_geometry(d, m, &r);
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;
    timing_events(&ev_begin, &ev_end);
    hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(64), 0, stream, ws->ctl);
    const unsigned init_blocks = (unsigned)std::max<long long>(
        1, std::min<long long>(((long long)n + 255) / 256, (long long)d.cus * 8));
    hipLaunchKernelGGL(k_init_labels, dim3(init_blocks), dim3(256), 0, stream, L, (unsigned)n,
                       r.warm ? 1 : 0, ws->ctl);
    CONTOUR_HIP(hipGetLastError());
    if (ev_begin) CONTOUR_HIP(hipEventRecord(ev_begin, stream));
    if (m > 0) {
        persistent_fn kp;
        sweep_fn ks;
        pick_kernels(r.block, r.ept, r.atomic || r.sync, &kp, &ks);
        const bool reorder = wants_reorder(r, m, n);
        Reorder ro;
        long long need = r.sync ? n : 0;
        if (reorder) {
            reorder_geometry(d, m, n, &ro);
            need += ro.elems;
        }
        if (need > 0) {
            int rc = workspace_scratch(ws, stream, need);
            if (rc) return rc;
        }
        if (reorder) {
            reorder_bind(&ro, ws->scratch);
            int rc = enqueue_reorder(ro, src, dst, stream);
            if (rc) return rc;
            src = ro.src2;
            dst = ro.dst2;
        }
        SolveArgs a;
        a.src = src;
        a.dst = dst;
        a.L = L;
        a.m = m;
        a.n = (unsigned)n;
        a.sched = r.sched;
        a.max_sweeps = r.max_sweeps;
        a.ctl = ws->ctl;
        a.watchdog = watchdog_ticks(d);
        a.win_cap = 0;
        a.win_shift = 0;
        a.win_margin = 0;
        const long long tile_edges = (long long)r.block * r.ept;
        const long long ntiles = (m + tile_edges - 1) / tile_edges;
        a.tiles_per_task = 1;
        a.tasks = ntiles;
        a.ntiles = ntiles;
        a.take = 1;
        const long long grid = r.grid ? r.grid : std::min<long long>(ntiles, (long long)d.cus * 16);
        int* other = r.sync ? ws->scratch + (reorder ? ro.elems : 0) : nullptr;
        int sweep = 0, ahead = 4;
        for (;;) {
            for (int i = 0; i < ahead; ++i, ++sweep) {
                const int* R = L;
                int* W = L;
                if (r.sync) {
                    R = (sweep & 1) ? other : L;
                    W = (sweep & 1) ? L : other;
                    hipLaunchKernelGGL(k_copy_labels, dim3(init_blocks), dim3(256), 0, stream, R, W,
                                       (unsigned)n, (const Ctl*)ws->ctl);
                }
                hipLaunchKernelGGL(ks, dim3((unsigned)grid), dim3(r.block), 0, stream, a, R, W, sweep);
            }
            CONTOUR_HIP(hipGetLastError());
            CONTOUR_HIP(hipMemcpyAsync(ws->host_ctl, ws->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream));
            CONTOUR_HIP(hipStreamSynchronize(stream));
            if (ws->host_ctl->state != ST_RUNNING) break;
            ahead = std::min(ahead * 2, 64);
        }
        // The final sweep of a converged synchronous solve changed nothing,
        // so L and L_u are equal and L already holds the result.  A solve
        // stopped by the sweep limit may end with the newer state in L_u.
        if (r.sync && ws->host_ctl->state != ST_CONVERGED && (ws->host_ctl->sweeps & 1))
            CONTOUR_HIP(hipMemcpyAsync(L, other, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, stream));
    }
    if (ev_end) CONTOUR_HIP(hipEventRecord(ev_end, stream));
    if (stats) {
        hipLaunchKernelGGL(k_write_stats, dim3(1), dim3(64), 0, stream, (const Ctl*)ws->ctl, stats, 0);
        CONTOUR_HIP(hipGetLastError());
    }
    return CONTOUR_OK;
}

static int run_solve(const int* src, const int* dst, long long m, int n, int* L, const Resolved& r,
                     contour_stats_t* stats, hipStream_t stream, unsigned long long* reads = nullptr)
{
    DeviceInfo d;
    int rc = device_info(&d);
    if (rc) return rc;
    Workspace* ws = nullptr;
    rc = workspace_for(stream, &ws);
    if (rc) return rc;
    if (r.driver == CONTOUR_DRIVER_HOSTLOOP) return run_hostloop(d, r, src, dst, m, n, L, ws, stats, stream);
    int* scratch = nullptr;
    if (m > 0 && wants_reorder(r, m, n)) {
        Reorder ro;
        solve_reorder_geometry(d, r, m, n, &ro);
        rc = workspace_scratch(ws, stream, ro.elems);
        if (rc) return rc;
        scratch = ws->scratch;
    }
    PersistentLaunch p;
    rc = prepare_persistent(d, r, src, dst, m, n, L, ws->ctl, scratch, &p);
    if (rc) return rc;
    p.args.reads = reads;
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;
    timing_events(&ev_begin, &ev_end);
    return enqueue_persistent(p, stats, stream, ev_begin, ev_end);
}

}  // namespace contour

extern "C" {

int contour_cc_ex(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t* labels_inout,
                  const contour_opts_t* opts, contour_stats_t* stats, contour_stream_t stream)
{
    if (m < 0 || n < 0) return CONTOUR_EINVAL;
    if (n > 0 && !labels_inout) return CONTOUR_EINVAL;
    if (m > 0 && (!src || !dst)) return CONTOUR_EINVAL;
    contour::Resolved r;
    int rc = contour::resolve_opts(opts, &r);
    if (rc) return rc;
    if (n == 0) {
        // No vertices: nothing to label.  Any edge would have an id outside
        // [0, 0), which the stats report without the edges being read.
        if (!stats) return CONTOUR_OK;
        contour::Workspace* ws = nullptr;
        rc = contour::workspace_for((hipStream_t)stream, &ws);
        if (rc) return rc;
        return contour::enqueue_empty_stats(ws->ctl, stats, m > 0 ? 1 : 0, (hipStream_t)stream);
    }
    return contour::run_solve(src, dst, m, n, labels_inout, r, stats, (hipStream_t)stream);
}

int contour_reserve(int64_t m, int32_t n, const contour_opts_t* opts, contour_stream_t stream)
{
    if (m < 0 || n < 0) return CONTOUR_EINVAL;
    contour::Resolved r;
    int rc = contour::resolve_opts(opts, &r);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    contour::Workspace* ws = nullptr;
    rc = contour::workspace_for(s, &ws);
    if (rc) return rc;
    if (n == 0 || m == 0) return CONTOUR_OK;
    contour::DeviceInfo d;
    rc = contour::device_info(&d);
    if (rc) return rc;
    // what run_solve, run_hostloop and contour_group_edges ask of the scratch
    long long need = r.sync ? n : 0;
    if (m < 0x7fffffffLL) {
        contour::Reorder ro;
        contour::solve_reorder_geometry(d, r, m, n, &ro);
        if (contour::wants_reorder(r, m, n)) need += ro.elems;
        contour::reorder_geometry(d, m, n, &ro);  // contour_group_edges: one pass
        need = std::max(need, contour::reorder_table_elems(ro));
    }
    return contour::workspace_scratch(ws, s, need);
}

int contour_cc_count_reads(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t* labels_inout,
                           const contour_opts_t* opts, contour_stats_t* stats, uint64_t* reads,
                           contour_stream_t stream)
{
    if (m < 0 || n < 0 || !reads) return CONTOUR_EINVAL;
    if (n > 0 && !labels_inout) return CONTOUR_EINVAL;
    if (m > 0 && (!src || !dst)) return CONTOUR_EINVAL;
    contour::Resolved r;
    int rc = contour::resolve_opts(opts, &r);
    if (rc) return rc;
    if (r.driver != CONTOUR_DRIVER_PERSISTENT) return CONTOUR_ENOTSUP;
    if (n == 0) return contour_cc_ex(src, dst, m, n, labels_inout, opts, stats, stream);
    return contour::run_solve(src, dst, m, n, labels_inout, r, stats, (hipStream_t)stream,
                              reinterpret_cast<unsigned long long*>(reads));
}

int contour_gather_ceiling(const int32_t* src, const int32_t* dst, int64_t m, const int32_t* labels, int32_t n,
                           int32_t mode, int32_t* sink, contour_stream_t stream)
{
    if (m < 0 || n < 0 || mode < 0 || mode > 2 || !sink) return CONTOUR_EINVAL;
    if (m > 0 && (!src || !dst)) return CONTOUR_EINVAL;
    if (mode > 0 && n > 0 && !labels) return CONTOUR_EINVAL;
    if (m == 0) return CONTOUR_OK;
    contour::DeviceInfo d;
    int rc = contour::device_info(&d);
    if (rc) return rc;
    // two resident 1024-thread workgroups per CU, four launched per CU
    const unsigned grid = (unsigned)std::max(8, (d.cus / 8) * 8 * 4);
    hipLaunchKernelGGL(contour::k_gather_ceiling, dim3(grid), dim3(1024), 0, (hipStream_t)stream, src, dst,
                       (long long)m, labels, (unsigned)n, mode, sink);
    CONTOUR_HIP(hipGetLastError());
    return CONTOUR_OK;
}

int contour_cc(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t* labels_out,
               contour_stream_t stream)
{
    return contour_cc_ex(src, dst, m, n, labels_out, nullptr, nullptr, stream);
}

int contour_group_edges(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t* src_out,
                        int32_t* dst_out, contour_stream_t stream)
{
    if (m < 0 || m >= 0x7fffffffLL || n <= 0) return CONTOUR_EINVAL;
    if (m == 0) return CONTOUR_OK;
    if (!src || !dst || !src_out || !dst_out) return CONTOUR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    contour::DeviceInfo d;
    int rc = contour::device_info(&d);
    if (rc) return rc;
    contour::Workspace* ws = nullptr;
    rc = contour::workspace_for(s, &ws);
    if (rc) return rc;
    contour::Reorder ro;
    contour::reorder_geometry(d, m, n, &ro);
    rc = contour::workspace_scratch(ws, s, contour::reorder_table_elems(ro));
    if (rc) return rc;
    contour::reorder_bind_tables(&ro, ws->scratch);
    ro.src2 = src_out;
    ro.dst2 = dst_out;
    return contour::enqueue_reorder(ro, src, dst, s);
}

int contour_group_edges_ranges(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t* src_out,
                               int32_t* dst_out, contour_stream_t stream)
{
    if (m < 0 || m >= 0x7fffffffLL || n <= (1 << contour::kDstRangeShift)) return CONTOUR_EINVAL;
    if (m == 0) return CONTOUR_OK;
    if (!src || !dst || !src_out || !dst_out) return CONTOUR_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    contour::DeviceInfo d;
    int rc = contour::device_info(&d);
    if (rc) return rc;
    contour::Workspace* ws = nullptr;
    rc = contour::workspace_for(s, &ws);
    if (rc) return rc;
    contour::Reorder ro;
    contour::reorder_geometry(d, m, n, &ro, contour::kDstRangeShift);
    // the first pass's copy and the count tables in the workspace, the
    // second pass writes the caller's arrays
    const long long mp = (m + 3) & ~3LL;
    rc = contour::workspace_scratch(ws, s, 2 * mp + contour::reorder_table_elems(ro));
    if (rc) return rc;
    ro.src1 = ws->scratch;
    ro.dst1 = ws->scratch + mp;
    contour::reorder_bind_tables(&ro, ws->scratch + 2 * mp);
    ro.src2 = src_out;
    ro.dst2 = dst_out;
    return contour::enqueue_reorder(ro, src, dst, s);
}

int contour_cc_add_edges(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t* labels_inout,
                         const contour_opts_t* opts, contour_stats_t* stats, contour_stream_t stream)
{
    if (m < 0 || n < 0) return CONTOUR_EINVAL;
    if (n > 0 && !labels_inout) return CONTOUR_EINVAL;
    if (m > 0 && (!src || !dst)) return CONTOUR_EINVAL;
    if (m > (0x7fffffffLL - 3) / 3) return CONTOUR_EINVAL;  // the augmented list has 3m edges
    contour::Resolved r;
    int rc = contour::resolve_opts(opts, &r);
    if (rc) return rc;
    r.warm = true;
    if (n == 0) return contour_cc_ex(src, dst, m, n, labels_inout, opts, stats, stream);
    hipStream_t s = (hipStream_t)stream;
    contour::Workspace* ws = nullptr;
    rc = contour::workspace_for(s, &ws);
    if (rc) return rc;
    const long long mp = (m + 3) & ~3LL;
    int* as = nullptr;
    int* ad = nullptr;
    if (m > 0) {
        // both arrays start on 16-byte boundaries
        rc = contour::workspace_aux(ws, s, 6 * mp);
        if (rc) return rc;
        as = ws->aux;
        ad = ws->aux + 3 * mp;
        contour::DeviceInfo d;
        rc = contour::device_info(&d);
        if (rc) return rc;
        const unsigned blocks = (unsigned)std::max<long long>(
            1, std::min<long long>((m + 255) / 256, (long long)d.cus * 8));
        hipLaunchKernelGGL(contour::k_tie_edges, dim3(blocks), dim3(256), 0, s, src, dst, (long long)m,
                           (const int*)labels_inout, (unsigned)n, as, ad);
        CONTOUR_HIP(hipGetLastError());
    }
    rc = contour::run_solve(as, ad, 3 * (long long)m, n, labels_inout, r, stats, s);
    if (rc) return rc;
    contour::DeviceInfo d;
    rc = contour::device_info(&d);
    if (rc) return rc;
    const unsigned blocks = (unsigned)std::max<long long>(
        1, std::min<long long>(((long long)n + 255) / 256, (long long)d.cus * 8));
    hipLaunchKernelGGL(contour::k_flatten, dim3(blocks), dim3(256), 0, s, labels_inout, (unsigned)n,
                       (const contour::Ctl*)ws->ctl);
    CONTOUR_HIP(hipGetLastError());
    return CONTOUR_OK;
}

}  // extern "C"
