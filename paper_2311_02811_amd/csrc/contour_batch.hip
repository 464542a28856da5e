// contour_batch.hip -- batched solve of many independent graphs in one plan.
//
// A batch is a CSR-of-graphs: graph g has local vertex ids 0..n_g-1 and its
// own edge range.  Each graph is solved exactly as a single graph would be
// (same operator, same convergence test); only the placement differs:
//   class 0  small graphs: one workgroup per graph, label array in LDS, the
//            whole solve inside the workgroup (barriers separate sweeps)
//   class 1  medium graphs: one workgroup per graph, labels in global memory
//            with the lowest ids of the graph held in LDS for the whole solve
//   class 2  large graphs: many workgroups per graph; one persistent kernel
//            spreads the workgroups over the graphs, each graph sequenced by
//            its own task counters (the single-graph persistent loop)
// Classes 0 and 1 take graphs from a queue ordered by decreasing edge count
// (longest first).  Class 1 runs on the caller's stream; class 2 and then
// class 0 run on a second stream concurrently with it.
// A launch enqueues kernels and event waits only, so it can be captured into
// a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "contour.h"
#include "contour_device.hpp"
#include "contour_persistent.hpp"
#include "contour_runtime.hpp"

namespace contour {

struct WgArgs {
    contour_stats_t* stats;  // [G] or null
    const BatchJob* jobs;
    int njobs;
    int* counter;  // queue position
    Sched sched;
    int max_sweeps;
    const Ctl* clock;  // t0 for the watchdog
    unsigned long long watchdog;
    int wcap;          // labels of a class-1 graph kept in LDS (the launch's dynamic LDS / 4; 0: none)
};

// Class-0 graphs up to this many vertices go to a launch whose workgroups
// hold 64 KiB of labels (two or more share a CU); larger class-0 graphs, up
// to the whole LDS of a CU, to a launch of their own.
static constexpr int kLdsSmall = 16384;

// ------------------------------------------------- one graph per workgroup --

// The sweeps of one graph inside one workgroup (barriers between sweeps);
// `global` when some labels live in global memory (stores drained before
// each barrier).  Returns the solve's state.
template <int EPT, int BLOCK, bool ATOMIC, class LAB>
__device__ __forceinline__ int wg_sweeps(const WgArgs& a, const BatchJob& job, const LAB& lab, bool global,
                                         int& sweep, int& last_change, int& rerr)
{
    const long long tile_edges = (long long)BLOCK * EPT;
    const long long ntiles = (job.m + tile_edges - 1) / tile_edges;
    if (job.m == 0) return ST_CONVERGED;
    for (;;) {
        const int order = order_of_sweep(a.sched, sweep);
        const bool pred = run_tiles_lab<EPT, BLOCK, ATOMIC>(job.src, job.dst, lab, 0, ntiles, 1, job.m,
                                                            (unsigned)job.n, order, rerr);
        if (global) drain_stores();
        const int any = uniform(__syncthreads_or(pred ? 1 : 0));
        ++sweep;
        if (!any) return ST_CONVERGED;
        last_change = sweep;
        if (a.max_sweeps > 0 && sweep >= a.max_sweeps) return ST_LIMIT;
        if ((sweep & 15) == 0) {
            const bool expired = watchdog_expired(a.clock, a.watchdog);
            if (uniform(__syncthreads_or(expired ? 1 : 0))) return ST_TIMEOUT;
        }
    }
}

// One graph in one workgroup.  MODE 0: every label in LDS (class 0); MODE 1:
// labels in global memory, the lowest a.wcap ids of them kept in LDS for the
// whole solve (class 1; without the window when a.wcap is 0 or n >= 2^30).
template <int EPT, int BLOCK, bool ATOMIC, int MODE>
__device__ __forceinline__ void wg_solve(const WgArgs& a, const BatchJob& job, int* lds)
{
    int sweep = 0, last_change = 0, rerr = 0, state;
    if (MODE == 0) {
        for (int i = threadIdx.x; i < job.n; i += BLOCK) lds[i] = i;
        __syncthreads();
        state = wg_sweeps<EPT, BLOCK, ATOMIC>(a, job, FlatLabels{lds, lds}, false, sweep, last_change, rerr);
        for (int i = threadIdx.x; i < job.n; i += BLOCK) job.labels[i] = lds[i];
    } else if (a.wcap > 0 && (unsigned)job.n < (1u << 30)) {
        const unsigned cnt = std::min((unsigned)job.n, (unsigned)a.wcap);
        for (unsigned i = threadIdx.x; i < cnt; i += BLOCK) lds[i] = (int)i;
        for (unsigned i = cnt + threadIdx.x; i < (unsigned)job.n; i += BLOCK) job.labels[i] = (int)i;
        drain_stores();
        __syncthreads();
        const OwnedWindowLabels lab{lds, cnt, job.labels, label_buffer(job.labels, (unsigned)job.n),
                                    (unsigned)job.n * 4u};
        state = wg_sweeps<EPT, BLOCK, ATOMIC>(a, job, lab, true, sweep, last_change, rerr);
        for (unsigned i = threadIdx.x; i < cnt; i += BLOCK) job.labels[i] = lds[i];
    } else {
        for (int i = threadIdx.x; i < job.n; i += BLOCK) job.labels[i] = i;
        drain_stores();
        __syncthreads();
        state = wg_sweeps<EPT, BLOCK, ATOMIC>(a, job, FlatLabels{job.labels, job.labels}, true, sweep,
                                              last_change, rerr);
    }
    const int anyerr = uniform(__syncthreads_or(rerr));
    if (a.stats && threadIdx.x == 0) {
        contour_stats_t st;
        st.status = anyerr ? CONTOUR_ERANGE : (state == ST_CONVERGED ? CONTOUR_OK : CONTOUR_ENOCONV);
        st.sweeps_executed = sweep;
        st.sweeps_with_writes = last_change;
        st.reserved = 0;
        a.stats[job.g] = st;
    }
}

template <int EPT, int BLOCK, bool ATOMIC, bool LDS>
__global__ __launch_bounds__(BLOCK) void k_batch_wg(WgArgs a)
{
    extern __shared__ int lds_labels[];
    __shared__ int s_job;
    if (threadIdx.x == 0) s_job = atomicAdd(a.counter, 1);
    __syncthreads();
    for (;;) {
        const int j = uniform(s_job);
        if (j >= a.njobs) break;
        const BatchJob job = a.jobs[j];
        wg_solve<EPT, BLOCK, ATOMIC, LDS ? 0 : 1>(a, job, lds_labels);
        __syncthreads();  // every lane has read s_job and finished with LDS
        if (threadIdx.x == 0) s_job = atomicAdd(a.counter, 1);
        __syncthreads();
    }
}

// --------------------------------------------- many workgroups per graph --

// Workgroups pick a graph: the first graph from the cursor on that is still
// running and has fewer than want[g] workgroups; when every graph has its
// share, a workgroup helps the first graph still running.  Inside a graph
// the persistent loop sequences the sweeps.  A workgroup exits when no
// graph is running.
__device__ __forceinline__ int multi_pick(const SolveArgs* graphs, int ngraphs, int* cursor, const int* want)
{
    int pick = -1;
    for (int g = __hip_atomic_load(cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); g < ngraphs; ++g) {
        Ctl* c = graphs[g].ctl;
        if (__hip_atomic_load(&c->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ST_RUNNING) {
            int e = g;
            __hip_atomic_compare_exchange_strong(cursor, &e, g + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        const int j = __hip_atomic_fetch_add(&c->joined, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (j < want[g]) {
            pick = g;
            break;
        }
    }
    if (pick < 0) {
        for (int g = __hip_atomic_load(cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); g < ngraphs; ++g) {
            if (__hip_atomic_load(&graphs[g].ctl->state, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ST_RUNNING) {
                pick = g;
                break;
            }
        }
    }
    return pick;
}

template <int EPT, int BLOCK, bool ATOMIC>
__global__ __launch_bounds__(BLOCK) void k_batch_multi(const SolveArgs* graphs, int ngraphs, int* cursor,
                                                       const int* want)
{
    __shared__ int s_g;
    if (threadIdx.x == 0) s_g = multi_pick(graphs, ngraphs, cursor, want);
    __syncthreads();
    for (;;) {
        const int g = uniform(s_g);
        if (g < 0) break;
        const SolveArgs a = graphs[g];
        persistent_solve<EPT, BLOCK, ATOMIC>(a);
        __syncthreads();  // every lane has read s_g
        if (threadIdx.x == 0) s_g = multi_pick(graphs, ngraphs, cursor, want);
        __syncthreads();
    }
}

// Reset the queue counters and the watchdog clock of a launch.
__global__ void k_batch_begin(int* counters, Ctl* clock)
{
    if (threadIdx.x < 4) counters[threadIdx.x] = 0;
    int* p = reinterpret_cast<int*>(clock);
    if (threadIdx.x < sizeof(Ctl) / sizeof(int)) p[threadIdx.x] = 0;
    __syncthreads();
    if (threadIdx.x == 0) clock->t0 = wall_clock64();
}

// Class-2 set-up: block (x, j) initialises part of graph j's labels; block
// (0, j) also resets graph j's control block.
__global__ void k_batch_multi_prepare(const SolveArgs* graphs)
{
    const SolveArgs& a = graphs[blockIdx.y];
    for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x)
        a.L[i] = (int)i;
    if (blockIdx.x == 0) {
        int* p = reinterpret_cast<int*>(a.ctl);
        if (threadIdx.x < sizeof(Ctl) / sizeof(int)) p[threadIdx.x] = 0;
        __syncthreads();
        if (threadIdx.x == 0) a.ctl->t0 = wall_clock64();
    }
}

__global__ void k_batch_multi_stats(const SolveArgs* graphs, const int* gidx, int ngraphs,
                                    contour_stats_t* stats)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ngraphs) return;
    const Ctl* c = graphs[j].ctl;
    contour_stats_t st;
    st.status = c->range_err ? CONTOUR_ERANGE
                             : ((c->state == ST_LIMIT || c->state == ST_TIMEOUT) ? CONTOUR_ENOCONV : CONTOUR_OK);
    st.sweeps_executed = c->sweeps;
    st.sweeps_with_writes = c->last_change;
    st.reserved = 0;
    stats[gidx[j]] = st;
}

// ------------------------------------------------------------- dispatch --

typedef void (*wg_fn)(WgArgs);
typedef void (*multi_fn)(const SolveArgs*, int, int*, const int*);

// 1024-thread workgroups with labels in global memory would spill registers
// at four edges per thread; they use two.
template <int BLOCK, bool ATOMIC, bool LDS>
static wg_fn pick_wg_e(int ept)
{
    switch (ept) {
    case 1: return k_batch_wg<1, BLOCK, ATOMIC, LDS>;
    case 2: return k_batch_wg<2, BLOCK, ATOMIC, LDS>;
    default: return k_batch_wg<(BLOCK == 1024 && !LDS) ? 2 : 4, BLOCK, ATOMIC, LDS>;
    }
}

template <bool ATOMIC, bool LDS>
static wg_fn pick_wg_b(int block, int ept)
{
    if (block == 1024) return pick_wg_e<1024, ATOMIC, LDS>(ept);
    if (block == 512) return pick_wg_e<512, ATOMIC, LDS>(ept);
    return pick_wg_e<256, ATOMIC, LDS>(ept);
}

static wg_fn pick_wg(int block, int ept, bool atomic, bool lds)
{
    if (atomic) return lds ? pick_wg_b<true, true>(block, ept) : pick_wg_b<true, false>(block, ept);
    return lds ? pick_wg_b<false, true>(block, ept) : pick_wg_b<false, false>(block, ept);
}

template <int BLOCK, bool ATOMIC>
static multi_fn pick_multi_e(int ept)
{
    switch (ept) {
    case 1: return k_batch_multi<1, BLOCK, ATOMIC>;
    case 2: return k_batch_multi<2, BLOCK, ATOMIC>;
    case 8: return k_batch_multi<8, BLOCK, ATOMIC>;
    default: return k_batch_multi<4, BLOCK, ATOMIC>;
    }
}

static multi_fn pick_multi(int block, int ept, bool atomic)
{
    if (block == 512) return atomic ? pick_multi_e<512, true>(ept) : pick_multi_e<512, false>(ept);
    return atomic ? pick_multi_e<256, true>(ept) : pick_multi_e<256, false>(ept);
}

static int wg_occupancy(wg_fn k, int block, size_t lds, int* occ)
{
    *occ = 0;
    CONTOUR_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, (const void*)k, block, lds));
    return CONTOUR_OK;
}

int enqueue_wg_jobs(const DeviceInfo& d, const Resolved& r, const BatchJob* d_jobs, int n_lds, int max_n_lds,
                    int n_global, int* d_counters, Ctl* d_clock, contour_stats_t* stats, hipStream_t stream)
{
    hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(64), 0, stream, d_counters, d_clock);
    const int counts[2] = {n_lds, n_global};
    for (int c = 1; c >= 0; --c) {
        if (counts[c] == 0) continue;
        const int block = r.block ? std::min(r.block, 1024) : 512;
        const int ept = r.ept ? std::min(r.ept, 4) : (c == 0 ? 1 : 2);
        WgArgs a;
        a.stats = stats;
        a.jobs = d_jobs + (c == 0 ? 0 : n_lds);
        a.njobs = counts[c];
        a.counter = d_counters + c;
        a.sched = r.sched;
        a.max_sweeps = r.max_sweeps;
        a.clock = d_clock;
        a.watchdog = watchdog_ticks(d);
        // class 1 keeps the lowest ids of each graph in the LDS (as in a plan)
        a.wcap = c == 1 ? std::max(0, (d.max_lds_per_block - 2048) / 4) & ~63 : 0;
        const wg_fn k = pick_wg(block, ept, r.atomic, c == 0);
        const size_t lds = c == 0 ? sizeof(int) * (size_t)std::max(max_n_lds, 1) : sizeof(int) * (size_t)a.wcap;
        if (lds > 0) (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        int occ = 0;
        int rc = wg_occupancy(k, block, lds, &occ);
        if (rc) return rc;
        const unsigned grid = (unsigned)std::min<long long>((long long)std::max(occ, 1) * d.cus, counts[c]);
        hipLaunchKernelGGL(k, dim3(grid), dim3(block), lds, stream, a);
        CONTOUR_HIP(hipGetLastError());
    }
    return CONTOUR_OK;
}

}  // namespace contour

// ----------------------------------------------------------------- plan --

struct contour_plan {
    int device = -1;
    int G = 0;
    int counts[3] = {0, 0, 0};
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int* d_counters = nullptr;         // queues: [0] class 0 (small LDS), [1] class 1, [3] class 0 (large
                                       // LDS); [2] class-2 cursor
    contour::Ctl* d_clock = nullptr;   // class 0/1 watchdog clock
    contour::BatchJob* d_jobs = nullptr;  // class 0 jobs then class 1 jobs
    contour::SolveArgs* d_graphs = nullptr;  // class 2
    contour::Ctl* d_ctl = nullptr;     // class 2 control blocks
    int* d_want = nullptr;
    int* d_gidx = nullptr;
    // one-workgroup launches: [0] class 0 up to kLdsSmall vertices, [1] class
    // 1, [2] class 0 above kLdsSmall vertices (the whole LDS of a CU)
    contour::WgArgs wg[3];
    contour::wg_fn wg_kernel[3] = {nullptr, nullptr, nullptr};
    unsigned wg_grid[3] = {0, 0, 0};
    int wg_block[3] = {256, 256, 256};
    size_t wg_lds[3] = {0, 0, 0};
    contour::multi_fn multi_kernel = nullptr;
    unsigned multi_grid = 0;
    int multi_block = 256;
    unsigned prep_x = 1;
    contour_stats_t* stats = nullptr;
};

namespace contour {

static void free_plan(contour_plan* p)
{
    if (!p) return;
    if (p->d_counters) (void)hipFree(p->d_counters);
    if (p->d_clock) (void)hipFree(p->d_clock);
    if (p->d_jobs) (void)hipFree(p->d_jobs);
    if (p->d_graphs) (void)hipFree(p->d_graphs);
    if (p->d_ctl) (void)hipFree(p->d_ctl);
    if (p->d_want) (void)hipFree(p->d_want);
    if (p->d_gidx) (void)hipFree(p->d_gidx);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->side) (void)hipStreamDestroy(p->side);
    delete p;
}

static int class_geometry(const contour_batch_tuning_t* t, int cls, int* block, int* ept, int* order,
                          int default_order)
{
    int b = t ? t->cls[cls].block : 0;
    int e = t ? t->cls[cls].edges_per_thread : 0;
    int o = t ? t->cls[cls].order : 0;
    if (t && t->cls[cls].reserved != 0) return CONTOUR_EINVAL;
    if (b == 0) b = cls == 2 ? 256 : 512;
    if (e == 0) e = cls == 0 ? 1 : (cls == 1 ? 2 : 4);
    if (o == 0) o = default_order;
    if (b != 256 && b != 512 && !(b == 1024 && cls < 2)) return CONTOUR_EINVAL;
    if (e != 1 && e != 2 && e != 4 && !(e == 8 && cls == 2)) return CONTOUR_EINVAL;
    if (!(o == CONTOUR_ORDER_FULL || (o >= 1 && o <= CONTOUR_ORDER_MAX))) return CONTOUR_EINVAL;
    *block = b;
    *ept = e;
    *order = o;
    return CONTOUR_OK;
}

template <typename T>
static hipError_t upload(T** dst, const std::vector<T>& v)
{
    *dst = nullptr;
    if (v.empty()) return hipSuccess;
    hipError_t e = hipMalloc((void**)dst, sizeof(T) * v.size());
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

static int create_plan(const contour_batch_t* b, const contour_opts_t* opts, const contour_batch_tuning_t* t,
                       contour_plan_t* out)
{
    if (!b || !out) return CONTOUR_EINVAL;
    *out = nullptr;
    const int G = b->num_graphs;
    if (G < 0 || (G > 0 && (!b->h_edge_offsets || !b->h_vertex_offsets))) return CONTOUR_EINVAL;
    Resolved r;
    int rc = resolve_opts(opts, &r);
    if (rc) return rc;
    if (r.sync || r.driver != CONTOUR_DRIVER_PERSISTENT || r.warm) return CONTOUR_ENOTSUP;
    const int64_t* eo = b->h_edge_offsets;
    const int64_t* vo = b->h_vertex_offsets;
    if (G > 0 && (eo[0] != 0 || vo[0] != 0)) return CONTOUR_EINVAL;
    for (int g = 0; g < G; ++g) {
        if (eo[g + 1] < eo[g] || vo[g + 1] < vo[g] || vo[g + 1] - vo[g] > 0x7fffffffLL) return CONTOUR_EINVAL;
    }
    const int64_t total_m = G ? eo[G] : 0, total_n = G ? vo[G] : 0;
    if (total_m > 0 && (!b->src || !b->dst)) return CONTOUR_EINVAL;
    if (total_n > 0 && !b->labels_out) return CONTOUR_EINVAL;

    DeviceInfo d;
    rc = device_info(&d);
    if (rc) return rc;
    int lds_max = t ? t->lds_max_vertices : 0;
    if (lds_max < 0) return CONTOUR_EINVAL;
    const int lds_cap = (d.max_lds_per_block - 1024) / 4;
    if (lds_max == 0 || lds_max > lds_cap) lds_max = lds_cap;
    long long wg_max = t ? t->wg_max_edges : 0;
    if (wg_max < 0) return CONTOUR_EINVAL;
    if (wg_max == 0) wg_max = 1 << 19;

    int block[3], ept[3], order[3];
    for (int c = 0; c < 3; ++c) {
        rc = class_geometry(t, c, &block[c], &ept[c], &order[c], r.sched.order);
        if (rc) return rc;
        // explicit (non-zero) options override the tuned choice, for every
        // class where the value is allowed
        if (opts && opts->order != 0) order[c] = r.sched.order;
        if (opts && opts->block != 0 && (opts->block != 1024 || c < 2)) block[c] = opts->block;
        if (opts && opts->edges_per_thread != 0 && (opts->edges_per_thread != 8 || c == 2))
            ept[c] = opts->edges_per_thread;
    }

    contour_plan* p = new (std::nothrow) contour_plan();
    if (!p) return CONTOUR_ENOMEM;
    p->G = G;
    p->stats = b->stats_out;
    CONTOUR_HIP(hipGetDevice(&p->device));

    // classify; longest graphs first within each class
    std::vector<int> idx(G);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
        return eo[x + 1] - eo[x] > eo[y + 1] - eo[y];
    });
    std::vector<BatchJob> jobs[3];  // per one-workgroup launch (see contour_plan::wg)
    std::vector<int> big;
    for (int g : idx) {
        BatchJob j;
        j.src = b->src + eo[g];
        j.dst = b->dst + eo[g];
        j.labels = b->labels_out + vo[g];
        j.m = eo[g + 1] - eo[g];
        j.n = (int)(vo[g + 1] - vo[g]);
        j.g = g;
        if (j.n <= lds_max)
            jobs[j.n <= kLdsSmall ? 0 : 2].push_back(j);
        else if (j.m <= wg_max)
            jobs[1].push_back(j);
        else
            big.push_back(g);
    }
    p->counts[0] = (int)(jobs[0].size() + jobs[2].size());
    p->counts[1] = (int)jobs[1].size();
    p->counts[2] = (int)big.size();

    hipError_t e = hipMalloc((void**)&p->d_counters, 4 * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void**)&p->d_clock, sizeof(Ctl));
    std::vector<BatchJob> all = jobs[0];
    all.insert(all.end(), jobs[1].begin(), jobs[1].end());
    all.insert(all.end(), jobs[2].begin(), jobs[2].end());
    if (e == hipSuccess) e = upload(&p->d_jobs, all);
    if (e != hipSuccess) {
        free_plan(p);
        return hip_fail(e);
    }
    const unsigned long long wd = watchdog_ticks(d);
    size_t first = 0;
    for (int u = 0; u < 3; ++u) {
        const int c = u == 1 ? 1 : 0;  // the class whose geometry the launch uses
        WgArgs& a = p->wg[u];
        a.stats = b->stats_out;
        a.jobs = p->d_jobs + first;
        a.njobs = (int)jobs[u].size();
        first += jobs[u].size();
        a.counter = p->d_counters + (u == 2 ? 3 : u);
        a.sched = r.sched;
        a.sched.order = order[c];
        a.max_sweeps = r.max_sweeps;
        a.clock = p->d_clock;
        a.watchdog = wd;
        int ub = block[c], ue = ept[c];
        if (u == 2) {
            // a large-LDS workgroup has its CU to itself: the largest
            // workgroup, four edges per thread
            ub = 1024;
            ue = 4;
        }
        p->wg_block[u] = ub;
        p->wg_kernel[u] = pick_wg(ub, ue, r.atomic, c == 0);
        int max_n = 0;
        for (const BatchJob& j : jobs[u]) max_n = std::max(max_n, j.n);
        p->wg_lds[u] = c == 0 ? sizeof(int) * (size_t)std::max(max_n, 1) : 0;
        a.wcap = 0;
        if (u == 1) {
            // class 1: the rest of the LDS keeps the lowest ids of the graph
            a.wcap = std::max(0, (d.max_lds_per_block - 2048) / 4) & ~63;
            p->wg_lds[u] = sizeof(int) * (size_t)a.wcap;
        }
        if (jobs[u].empty()) continue;
        if (u == 1 && a.wcap > 0)
            (void)hipFuncSetAttribute((const void*)p->wg_kernel[u], hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)p->wg_lds[u]);
        if (c == 0) {
            // launches 0 and 2 share the kernel: allow the larger of the two
            const size_t most = std::max(p->wg_lds[0], u == 2 ? p->wg_lds[2] : 0);
            (void)hipFuncSetAttribute((const void*)p->wg_kernel[u], hipFuncAttributeMaxDynamicSharedMemorySize,
                                      (int)most);
        }
        int occ = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)p->wg_kernel[u], ub,
                                                         p->wg_lds[u]);
        if (e != hipSuccess) {
            free_plan(p);
            return hip_fail(e);
        }
        p->wg_grid[u] = (unsigned)std::max<long long>(
            0, std::min<long long>((long long)std::max(occ, 1) * d.cus, (long long)jobs[u].size()));
    }

    // a side stream for class 2 and class 0 (default priority, like the
    // caller's), joined back by an event
    if (!big.empty() || (!jobs[1].empty() && jobs[0].size() + jobs[2].size() > 0)) {
        e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
        if (e != hipSuccess) {
            free_plan(p);
            return hip_fail(e);
        }
    }
    if (!big.empty()) {
        std::vector<Ctl> zero(big.size());
        std::memset(zero.data(), 0, sizeof(Ctl) * zero.size());
        e = upload(&p->d_ctl, zero);
        std::vector<SolveArgs> graphs;
        std::vector<int> want;
        Resolved rc2 = r;
        rc2.sched.order = order[2];
        rc2.block = block[2];
        rc2.ept = ept[2];
        rc2.grid = 0;
        rc2.reorder = CONTOUR_REORDER_OFF;
        rc2.solo = false;
        p->multi_kernel = pick_multi(block[2], ept[2], r.atomic);
        int occ = 0;
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)p->multi_kernel, block[2], 0);
        const long long resident = (long long)std::max(occ, 1) * d.cus;
        long long sum_want = 0;
        unsigned max_n = 1;
        for (size_t k = 0; e == hipSuccess && k < big.size(); ++k) {
            const int g = big[k];
            PersistentLaunch pl;
            int rr = prepare_persistent(d, rc2, b->src + eo[g], b->dst + eo[g], eo[g + 1] - eo[g],
                                        (int)(vo[g + 1] - vo[g]), b->labels_out + vo[g], p->d_ctl + k, nullptr, &pl);
            if (rr) {
                free_plan(p);
                return rr;
            }
            long long w = std::max<long long>(1, std::min<long long>(resident, (pl.args.tasks + 3) / 4));
            pl.args.take = (int)std::max<long long>(1, pl.args.tasks / w);
            graphs.push_back(pl.args);
            want.push_back((int)w);
            sum_want += w;
            max_n = std::max(max_n, pl.args.n);
        }
        if (e == hipSuccess) e = upload(&p->d_graphs, graphs);
        if (e == hipSuccess) e = upload(&p->d_want, want);
        if (e == hipSuccess) e = upload(&p->d_gidx, big);
        if (e != hipSuccess) {
            free_plan(p);
            return hip_fail(e);
        }
        p->multi_block = block[2];
        p->multi_grid = (unsigned)std::min<long long>(resident, sum_want);
        p->prep_x = (unsigned)std::max<long long>(1, std::min<long long>(((long long)max_n + 255) / 256, 1024));
    }
    *out = p;
    return CONTOUR_OK;
}

static int launch_plan(contour_plan* p, hipStream_t stream)
{
    if (!p) return CONTOUR_EINVAL;
    if (p->G == 0) return CONTOUR_OK;
    hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(64), 0, stream, p->d_counters, p->d_clock);
    CONTOUR_HIP(hipGetLastError());
    const int nbig = p->counts[2];
    // Class 1 (the longest queue of one-workgroup solves) runs on the
    // caller's stream; class 2 and then class 0 (large LDS first) run on the
    // side stream beside it.  A class-1 workgroup leaves room on its CU for
    // class-0 workgroups, so class 0 is taken off the critical path.
    const bool fork = p->side && (nbig > 0 || (p->wg_grid[1] && (p->wg_grid[0] || p->wg_grid[2])));
    if (fork) {
        CONTOUR_HIP(hipEventRecord(p->ev_fork, stream));
        CONTOUR_HIP(hipStreamWaitEvent(p->side, p->ev_fork, 0));
    }
    if (nbig > 0) {
        hipLaunchKernelGGL(k_batch_multi_prepare, dim3(p->prep_x, nbig), dim3(256), 0, p->side,
                           (const SolveArgs*)p->d_graphs);
        hipLaunchKernelGGL(p->multi_kernel, dim3(p->multi_grid), dim3(p->multi_block), 0, p->side,
                           (const SolveArgs*)p->d_graphs, nbig, p->d_counters + 2, (const int*)p->d_want);
        if (p->stats)
            hipLaunchKernelGGL(k_batch_multi_stats, dim3((nbig + 63) / 64), dim3(64), 0, p->side,
                               (const SolveArgs*)p->d_graphs, (const int*)p->d_gidx, nbig, p->stats);
        CONTOUR_HIP(hipGetLastError());
    }
    for (int u : {1, 2, 0}) {
        if (p->wg_grid[u] == 0) continue;
        hipLaunchKernelGGL(p->wg_kernel[u], dim3(p->wg_grid[u]), dim3(p->wg_block[u]), p->wg_lds[u],
                           u != 1 && fork ? p->side : stream, p->wg[u]);
        CONTOUR_HIP(hipGetLastError());
    }
    if (fork) {
        CONTOUR_HIP(hipEventRecord(p->ev_join, p->side));
        CONTOUR_HIP(hipStreamWaitEvent(stream, p->ev_join, 0));
    }
    return CONTOUR_OK;
}

}  // namespace contour

extern "C" {

int contour_batch_plan_create_tuned(const contour_batch_t* batch, const contour_opts_t* opts,
                                    const contour_batch_tuning_t* tuning, contour_plan_t* plan_out)
{
    return contour::create_plan(batch, opts, tuning, plan_out);
}

int contour_batch_plan_create(const contour_batch_t* batch, const contour_opts_t* opts, contour_plan_t* plan_out)
{
    return contour::create_plan(batch, opts, nullptr, plan_out);
}

int contour_batch_plan_classes(contour_plan_t plan, int32_t* counts)
{
    if (!plan || !counts) return CONTOUR_EINVAL;
    for (int c = 0; c < 3; ++c) counts[c] = plan->counts[c];
    return CONTOUR_OK;
}

int contour_batch_plan_launch(contour_plan_t plan, contour_stream_t stream)
{
    return contour::launch_plan(plan, (hipStream_t)stream);
}

int contour_batch_plan_destroy(contour_plan_t plan)
{
    if (!plan) return CONTOUR_OK;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && dev == plan->device) (void)hipDeviceSynchronize();
    contour::free_plan(plan);
    return CONTOUR_OK;
}

int contour_cc_batched(const contour_batch_t* batch, const contour_opts_t* opts, contour_stream_t stream)
{
    contour_plan_t p = nullptr;
    int rc = contour::create_plan(batch, opts, nullptr, &p);
    if (rc) return rc;
    rc = contour::launch_plan(p, (hipStream_t)stream);
    if (rc == CONTOUR_OK) {
        hipError_t e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) rc = contour::hip_fail(e);
    }
    contour::free_plan(p);
    return rc;
}

}  // extern "C"
