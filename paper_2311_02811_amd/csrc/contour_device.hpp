// contour_device.hpp -- device-side building blocks of the Contour sweep.
//
// One edge <w, v> under the h-order minimum-mapping operator MM^h
// (Definition 3): read the chains x_0 = w, x_1 = L[x_0], ..., x_h and
// y_0 = v, ..., y_h, take z = min(x_h, y_h), and for i < h store z into
// L[x_i] (resp. L[y_i]) when the value read there, x_{i+1}, exceeds z
// (conditional assignment, Definition 1).  A chain stops early at a root
// (L[x] = x): deeper levels would only repeat it.
//
// Every label array the kernels touch satisfies L[x] <= x at every instant
// (it holds initially, and a store only ever lowers a value it read to a
// smaller label of the same component), so each chain is non-increasing and
// the edge changes something exactly when max(x_1, y_1) > z.  That is the
// early convergence test of Section III-B-2 (for h >= 2 it is the paper's
// L[v] != L^2[v] || L[w] != L^2[w] || L[v] != L[w]), and it is evaluated on
// the values read before the edge's own stores.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace contour {

// Per-solve control block (one per graph in a batch), 128 bytes.
struct Ctl {
    unsigned long long next_task;  // persistent driver: next task index to hand out
    unsigned long long done_task;  // persistent driver: tasks completed
    int last_change;               // 1 + index of the last sweep in which an edge changed a label
    int state;                     // 0 running, 1 converged, 2 sweep limit, 3 bad warm start
    int range_err;                 // an edge had an id outside [0, n)
    int sweeps;                    // sweeps executed (set when the solve ends)
    int joined;                    // batched multi-workgroup graphs: workgroups that joined
    int pad[3];
    unsigned long long t0;         // wall clock at the start of the solve (watchdog)
    unsigned long long pad2;
    unsigned long long xq[8];      // persistent driver, XCD queues: units taken from each XCD's segment
};
static_assert(sizeof(Ctl) == 128, "control block is two 64-byte lines");

enum { ST_RUNNING = 0, ST_CONVERGED = 1, ST_LIMIT = 2, ST_BAD_START = 3, ST_TIMEOUT = 4 };

// Watchdog: a solve that runs longer than its time budget (measured with the
// constant-rate wall clock) stops as if it had hit the sweep limit, so no
// kernel can spin forever whatever the input.
__device__ __forceinline__ bool watchdog_expired(const Ctl* c, unsigned long long budget)
{
    return budget != 0 && wall_clock64() - c->t0 > budget;
}

// Operator schedule (Section III-B-4): order of MM^h used in a given sweep.
struct Sched {
    int order;  // 1..1024, or -1 for chase-to-root
    int kind;   // 0 fixed, 1 C-11mm, 2 C-1m1m
    int k1;     // C-11mm: sweeps of order 1 first
};

__device__ __forceinline__ int order_of_sweep(const Sched& s, int sweep)
{
    if (s.kind == 1) return sweep < s.k1 ? 1 : s.order;
    if (s.kind == 2) return (sweep & 1) ? s.order : 1;
    return s.order;
}

// Arguments of one single-graph solve.
struct SolveArgs {
    const int* src;
    const int* dst;
    int* L;
    long long m;
    unsigned n;
    long long tasks;     // persistent driver: tasks per sweep
    long long ntiles;    // persistent driver: tiles of BLOCK * EPT edges per sweep
    int tiles_per_task;  // persistent driver: the largest task, in tiles
    int take;            // persistent driver: tasks a workgroup takes at once (>= 1)
    Sched sched;
    int max_sweeps;      // 0 = no limit
    Ctl* ctl;
    unsigned long long watchdog;  // wall-clock ticks a solve may run, 0 = unbounded
    int win_cap;         // LDS window capacity in labels (0: no window)
    int win_shift;       // edges are grouped by src >> win_shift
    int win_margin;      // labels staged past the last source block of a task
    int xq_units;        // persistent driver: 0, one task counter for the whole GPU; else
                         // per-XCD queues of xq_units strided task groups per sweep
    unsigned long long* reads = nullptr;  // instrumented solve: label reads of orders above 3
                                          // (and chase-to-root) are added here; else null
};

// Edge ids are streamed once per sweep: non-temporal loads keep them from
// displacing the label array in the caches.
__device__ __forceinline__ int ld_edge(const int* p) { return __builtin_nontemporal_load(p); }

template <bool ATOMIC>
__device__ __forceinline__ void put(int* L, int x, int z)
{
    if (ATOMIC)
        __hip_atomic_fetch_min(L + x, z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        L[x] = z;
}

// Atomic minimum of z into L[x] from the active lanes of a wave, where many
// lanes often target the same label with the same value (a component's root
// late in a solve): lanes equal in both to the first active lane leave the
// atomic to that lane.  Exact: the minimum is the same, with fewer atomics on
// one address.
__device__ __forceinline__ void put_min_shared(int* L, int x, int z)
{
    const int x0 = __builtin_amdgcn_readfirstlane(x);
    const int z0 = __builtin_amdgcn_readfirstlane(z);
    const unsigned long long active = __builtin_amdgcn_ballot_w64(true);
    const bool leader = (int)__lane_id() == __builtin_ctzll(active);
    if (leader || x != x0 || z != z0)
        __hip_atomic_fetch_min(L + x, z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// Edge tile: BLOCK * EPT consecutive edges starting at `base`, EPT per
// thread, read so that every load instruction of a wave covers contiguous
// bytes.  All first-level gathers of a thread are issued
// before any second-level gather, and all gathers before any store.
// R is the array read, W the array written; they are the same array for the
// asynchronous update and differ for the synchronous one (Algorithm 1).
// Returns whether any of the thread's edges changed something; sets *rerr
// when an edge id is outside [0, n) (that edge is skipped).
// ---------------------------------------------------------------------------

typedef int edge2_t __attribute__((ext_vector_type(2)));
typedef int edge4_t __attribute__((ext_vector_type(4)));

template <int EPT, int BLOCK>
__device__ __forceinline__ void fetch_tile(const int* __restrict__ src, const int* __restrict__ dst,
                                           long long base, long long m, int (&w)[EPT], int (&v)[EPT],
                                           bool (&ok)[EPT])
{
    // A whole tile with 8- or 16-byte aligned arrays: thread t takes EPT
    // consecutive edges with one vector load per array (fewer memory
    // instructions for the address unit to process).  Both conditions are
    // the same for every lane.
    constexpr int VW = EPT % 4 == 0 ? 4 : EPT % 2 == 0 ? 2 : 1;
    if (VW > 1 && base + (long long)BLOCK * EPT <= m &&
        ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & (VW * 4 - 1)) == 0) {
        const long long e0 = base + (long long)threadIdx.x * EPT;
#pragma unroll
        for (int j = 0; j < EPT / VW; ++j) {
            if (VW == 4) {
                const edge4_t a = __builtin_nontemporal_load(reinterpret_cast<const edge4_t*>(src + e0) + j);
                const edge4_t b = __builtin_nontemporal_load(reinterpret_cast<const edge4_t*>(dst + e0) + j);
                w[4 * j] = a.x, w[4 * j + 1] = a.y, w[4 * j + 2] = a.z, w[4 * j + 3] = a.w;
                v[4 * j] = b.x, v[4 * j + 1] = b.y, v[4 * j + 2] = b.z, v[4 * j + 3] = b.w;
            } else {
                const edge2_t a = __builtin_nontemporal_load(reinterpret_cast<const edge2_t*>(src + e0) + j);
                const edge2_t b = __builtin_nontemporal_load(reinterpret_cast<const edge2_t*>(dst + e0) + j);
                w[2 * j] = a.x, w[2 * j + 1] = a.y;
                v[2 * j] = b.x, v[2 * j + 1] = b.y;
            }
        }
#pragma unroll
        for (int k = 0; k < EPT; ++k) ok[k] = true;
        return;
    }
    // Otherwise thread t takes edges base + k * BLOCK + t.  Loads are
    // unconditional (an edge past the end re-reads edge m-1) so that every
    // load of the tile is in flight at once instead of each waiting behind a
    // branch.
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const long long e = base + (long long)k * BLOCK + threadIdx.x;
        ok[k] = e < m;
        const long long ec = ok[k] ? e : m - 1;
        w[k] = ld_edge(src + ec);
        v[k] = ld_edge(dst + ec);
    }
}

// Range check: an edge with an id outside [0, n) is flagged and skipped (it
// then gathers label 0 and stores nothing).
template <int EPT>
__device__ __forceinline__ void check_tile(unsigned n, int (&w)[EPT], int (&v)[EPT], bool (&ok)[EPT], int& rerr)
{
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const bool inr = (unsigned)w[k] < n && (unsigned)v[k] < n;
        if (ok[k] && !inr) rerr = 1;
        ok[k] = ok[k] && inr;
        w[k] = ok[k] ? w[k] : 0;
        v[k] = ok[k] ? v[k] : 0;
    }
}

// MM^1: z = min(L[w], L[v]); targets w, v.
template <int EPT, bool ATOMIC, class LAB>
__device__ __forceinline__ bool tile_order1(const LAB& lab, const int (&w)[EPT],
                                            const int (&v)[EPT], const bool (&ok)[EPT])
{
    int a[EPT], b[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        a[k] = lab.ld(w[k]);
        b[k] = lab.ld(v[k]);
    }
    bool pred = false;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int z = min(a[k], b[k]);
        const bool act = ok[k] && max(a[k], b[k]) > z;
        pred |= act;
        if (act && a[k] > z) lab.template st<ATOMIC>(w[k], z);
        if (act && b[k] > z) lab.template st<ATOMIC>(v[k], z);
    }
    return pred;
}

// MM^2: z = min(L[L[w]], L[L[v]]); targets w, v, L[w], L[v].
template <int EPT, bool ATOMIC, class LAB>
__device__ __forceinline__ bool tile_order2(const LAB& lab, const int (&w)[EPT],
                                            const int (&v)[EPT], const bool (&ok)[EPT])
{
    int a[EPT], b[EPT], a2[EPT], b2[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        a[k] = lab.ld(w[k]);
        b[k] = lab.ld(v[k]);
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        a2[k] = lab.ld(a[k]);
        b2[k] = lab.ld(b[k]);
    }
    bool pred = false;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int z = min(a2[k], b2[k]);
        const bool act = ok[k] && max(a[k], b[k]) > z;
        pred |= act;
        if (act && a[k] > z) lab.template st<ATOMIC>(w[k], z);
        if (act && a2[k] > z) lab.template st<ATOMIC>(a[k], z);
        if (act && b[k] > z) lab.template st<ATOMIC>(v[k], z);
        if (act && b2[k] > z) lab.template st<ATOMIC>(b[k], z);
    }
    return pred;
}

// MM^3: z = min(L^3[w], L^3[v]); targets w, L[w], L^2[w] and the same for v.
template <int EPT, bool ATOMIC, class LAB>
__device__ __forceinline__ bool tile_order3(const LAB& lab, const int (&w)[EPT],
                                            const int (&v)[EPT], const bool (&ok)[EPT])
{
    int a[EPT], b[EPT], a2[EPT], b2[EPT], a3[EPT], b3[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        a[k] = lab.ld(w[k]);
        b[k] = lab.ld(v[k]);
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        a2[k] = lab.ld(a[k]);
        b2[k] = lab.ld(b[k]);
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        a3[k] = lab.ld(a2[k]);
        b3[k] = lab.ld(b2[k]);
    }
    bool pred = false;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int z = min(a3[k], b3[k]);
        const bool act = ok[k] && max(a[k], b[k]) > z;
        pred |= act;
        if (act && a[k] > z) lab.template st<ATOMIC>(w[k], z);
        if (act && a2[k] > z) lab.template st<ATOMIC>(a[k], z);
        if (act && a3[k] > z) lab.template st<ATOMIC>(a2[k], z);
        if (act && b[k] > z) lab.template st<ATOMIC>(v[k], z);
        if (act && b2[k] > z) lab.template st<ATOMIC>(b[k], z);
        if (act && b3[k] > z) lab.template st<ATOMIC>(b2[k], z);
    }
    return pred;
}

// MM^h for any h >= 1 (h < 0: chase to the root).  First walk: read both
// chains level by level (all of a thread's edges advance together) until
// level h or the root.  Second walk, only for edges that change something:
// from each endpoint again, store z where the value read exceeds z, stopping
// at level h, at the root, or where the value read is already <= z (the rest
// of a non-increasing chain is then <= z too).  The second walk re-reads the
// chain; any value it reads is a valid label, and if its reads differ from
// the first walk's, some other edge stored in this sweep, so a sweep that
// reports a change always makes one.
//
// nread (may be null) counts the label reads of the first walk: the reads
// that MM^h prescribes (levels 1..h, or up to the root), for measuring the
// chase-to-root operator's traffic.
template <int EPT, bool ATOMIC, class LAB>
__device__ __forceinline__ bool tile_orderh(const LAB& lab, const int (&w)[EPT],
                                            const int (&v)[EPT], const bool (&ok)[EPT], int h,
                                            int* nread = nullptr)
{
    int cw[EPT], cv[EPT], fw[EPT], fv[EPT];
    bool dw[EPT], dv[EPT];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        cw[k] = w[k];
        cv[k] = v[k];
        fw[k] = w[k];
        fv[k] = v[k];
        dw[k] = !ok[k];
        dv[k] = !ok[k];
    }
    for (int lvl = 0; h < 0 || lvl < h; ++lvl) {
        bool more = false;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
            int nw = cw[k], nv = cv[k];
            if (!dw[k]) nw = lab.ld(cw[k]);
            if (!dv[k]) nv = lab.ld(cv[k]);
            if (nread) *nread += (dw[k] ? 0 : 1) + (dv[k] ? 0 : 1);
            if (lvl == 0) {
                fw[k] = nw;
                fv[k] = nv;
            }
            if (!dw[k]) {
                if (nw == cw[k]) dw[k] = true;
                cw[k] = nw;
            }
            if (!dv[k]) {
                if (nv == cv[k]) dv[k] = true;
                cv[k] = nv;
            }
            more |= !dw[k] || !dv[k];
        }
        if (!more) break;
    }
    bool pred = false;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        if (!ok[k]) continue;
        int z = min(cw[k], cv[k]);
        if (max(fw[k], fv[k]) <= z) continue;
        pred = true;
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            int x = side ? v[k] : w[k];
            for (int lvl = 0; h < 0 || lvl < h; ++lvl) {
                int val = lab.ld(x);
                if (val > z) lab.template st<ATOMIC>(x, z);
                if (val <= z || val == x) break;
                x = val;
            }
        }
    }
    return pred;
}

// Apply MM^ORDER (ORDER 0: the run-time order h) to the tiles
// first, first + stride, ... (count of them), stopping at m.  The edges of
// the next DEPTH-1 tiles are in flight while a tile is processed (a ring of
// register slots, unrolled so that every slot index is a constant), so the
// edge stream's latency overlaps the label gathers.
template <int ORDER, int EPT, int BLOCK, bool ATOMIC, class LAB, int DEPTH = 4>
__device__ __forceinline__ bool run_tiles(const int* __restrict__ src, const int* __restrict__ dst,
                                          const LAB& lab, long long first, long long count,
                                          long long stride, long long m, unsigned n, int h, int& rerr,
                                          int* nread = nullptr)
{
    const long long tile_edges = (long long)BLOCK * EPT;
    const long long step = stride * tile_edges;
    long long base = first * tile_edges;
    if (count <= 0 || base >= m) return false;
    bool pred = false;
    int w[DEPTH][EPT], v[DEPTH][EPT];
    bool ok[DEPTH][EPT];
#pragma unroll
    for (int d = 0; d < DEPTH - 1; ++d) fetch_tile<EPT, BLOCK>(src, dst, base + d * step, m, w[d], v[d], ok[d]);
    bool done = false;
    for (long long i = 0; i < count && !done; i += DEPTH) {
#pragma unroll
        for (int d = 0; d < DEPTH; ++d) {
            const long long tb = base + (long long)d * step;
            if (i + d >= count || tb >= m) {
                done = true;
                break;
            }
            // refill the slot freed one round ago with tile i + d + DEPTH - 1
            constexpr int ahead = DEPTH - 1;
            const int slot = (d + ahead) % DEPTH;
            fetch_tile<EPT, BLOCK>(src, dst, tb + ahead * step, m, w[slot], v[slot], ok[slot]);
            check_tile<EPT>(n, w[d], v[d], ok[d], rerr);
            if (ORDER == 1) pred |= tile_order1<EPT, ATOMIC>(lab, w[d], v[d], ok[d]);
            else if (ORDER == 2) pred |= tile_order2<EPT, ATOMIC>(lab, w[d], v[d], ok[d]);
            else if (ORDER == 3) pred |= tile_order3<EPT, ATOMIC>(lab, w[d], v[d], ok[d]);
            else pred |= tile_orderh<EPT, ATOMIC>(lab, w[d], v[d], ok[d], h, nread);
        }
        base += (long long)DEPTH * step;
    }
    return pred;
}

// Prefetch depth: tiles of edges in flight per thread, chosen so that the
// registers fit the workgroup size (128 per lane at 1024 threads, 256 at 512)
// without spilling.
template <int EPT, int BLOCK>
struct TileDepth {
    static constexpr int value = BLOCK == 1024 ? (EPT == 1 ? 4 : EPT == 2 ? 2 : 1) : (EPT <= 2 ? 4 : 2);
};

template <int EPT, int BLOCK, bool ATOMIC, class LAB, int DEPTH = TileDepth<EPT, BLOCK>::value>
__device__ __forceinline__ bool run_tiles_lab(const int* __restrict__ src, const int* __restrict__ dst,
                                              const LAB& lab, long long first, long long count,
                                              long long stride, long long m, unsigned n, int h, int& rerr,
                                              int* nread = nullptr)
{
    switch (h) {
    case 1: return run_tiles<1, EPT, BLOCK, ATOMIC, LAB, DEPTH>(src, dst, lab, first, count, stride, m, n, h, rerr);
    case 2: return run_tiles<2, EPT, BLOCK, ATOMIC, LAB, DEPTH>(src, dst, lab, first, count, stride, m, n, h, rerr);
    case 3: return run_tiles<3, EPT, BLOCK, ATOMIC, LAB, DEPTH>(src, dst, lab, first, count, stride, m, n, h, rerr);
    default:
        // A chain strictly decreases until its root, so it has at most n
        // vertices: chase-to-root is the order n operator, and the bound also
        // caps every walk.
        if (h < 0 || (unsigned)h > n) h = (int)n;
        return run_tiles<0, EPT, BLOCK, ATOMIC, LAB, DEPTH>(src, dst, lab, first, count, stride, m, n, h, rerr,
                                                            nread);
    }
}

// Labels read from R and written to W, both in global memory (or both the
// same LDS array for a graph solved inside one workgroup).
struct FlatLabels {
    const int* R;
    int* W;
    __device__ __forceinline__ int ld(int x) const { return R[x]; }
    template <bool ATOMIC>
    __device__ __forceinline__ void st(int x, int z) const { put<ATOMIC>(W, x, z); }
};

// A window of the label array, ids [lo, lo + cnt), staged in LDS; ids
// outside it are read and written in global memory G.  The workgroup writes
// the labels it lowered in the window back once at the end of its task.
// Which ones those are is kept in the labels themselves: every staged label
// carries the tag bit kLabelClean (labels are below 2^30 wherever windows are
// used), a store into the window writes the untagged value, and a read masks
// the tag off.  A store thus needs no second LDS operation to mark it, and a
// smaller value always replaces a staged one under an atomic minimum too
// (the tagged value is larger than any label).
//
// A gather issues an LDS read (clamped index) and, unless every lane of the
// wave reads inside the window, a buffer load of G whose offset is pushed out
// of the buffer's range for the lanes inside the window: the hardware range
// check turns those lanes into no-ops that return 0, and a select keeps the
// right value.  The only branch is wave-uniform, so all gathers of a tile
// stay in flight together, and a wave whose gathers all hit the window waits
// on LDS only, not behind its own edge prefetches (vector memory loads
// complete in order).  An ordinary load of G under a per-lane branch would
// be merged with the LDS read into one flat load, or write the same register
// and wait for it.  Buffer offsets are 32-bit bytes, so label windows are
// only used for n < 2^30 (a host-side rule).
constexpr unsigned kBufferDataFormat32 = 4u << 15;  // buffer resource word 3: 32-bit elements
constexpr int kLabelClean = 1 << 30;                // tag of a staged, unchanged window label

__device__ __forceinline__ __amdgpu_buffer_rsrc_t label_buffer(const int* G, unsigned n)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<int*>(G), (short)0, (int)(n * 4u),
                                             (int)kBufferDataFormat32);
}

// Stores outside the window go to a small hash table in LDS (kHubSlots
// entries of id and minimum value), flushed to global memory with one
// atomic minimum per entry at the end of the task: late in a solve most of
// them hook the same few component roots, which would otherwise take an
// atomic in memory per edge.  An id whose slot is held by another id takes
// the global atomic directly.
constexpr int kHubSlots = 1024;

__device__ __forceinline__ unsigned hub_slot(int x)
{
    return ((unsigned)x * 2654435761u) >> (32 - 10);  // kHubSlots = 2^10
}

struct WindowLabels {
    int* lds;
    unsigned lo;
    unsigned cnt;
    int* G;
    __amdgpu_buffer_rsrc_t rsrc;
    unsigned oob;  // a byte offset past the end of G: 4 n
    int* hkey;     // LDS hub table: ids (-1: free) ...
    int* hval;     // ... and the smallest value stored to each
    __device__ __forceinline__ int ld(int x) const
    {
        typedef __attribute__((address_space(3))) const int* lds_ptr;
        const unsigned i = (unsigned)x - lo;
        const bool in = i < cnt;
        const int vl = ((lds_ptr)lds)[in ? i : 0];
        int vg = 0;
        if (__builtin_amdgcn_ballot_w64(!in) != 0)  // wave-uniform: skipped when every id is in the window
            vg = __builtin_amdgcn_raw_buffer_load_b32(rsrc, in ? oob : (unsigned)x * 4u, 0, 0);
        return in ? (vl & (kLabelClean - 1)) : vg;
    }
    template <bool ATOMIC>
    __device__ __forceinline__ void st(int x, int z) const
    {
        const unsigned i = (unsigned)x - lo;
        if (i < cnt) {
            if (ATOMIC)
                atomicMin(&lds[i], z);
            else
                lds[i] = z;
        } else {
            const unsigned h = hub_slot(x);
            const int k = atomicCAS(&hkey[h], -1, x);
            if (k == -1 || k == x)
                atomicMin(&hval[h], z);
            else
                put_min_shared(G, x, z);  // global memory: atomic minimum (see persistent_solve)
        }
    }
};

// The labels of a graph that one workgroup owns for its whole solve: ids
// [0, cnt) in LDS, the rest in global memory G.  No other workgroup touches
// them, so a store outside the window goes to G directly (by the write
// mode), and the caller writes the window back when the solve ends.  Labels
// move towards the smallest ids of their components, so after the first
// sweep most of the deeper gathers of a chain land in the window.  Gathers
// as in WindowLabels (LDS read plus a range-checked buffer load skipped when
// the whole wave hits the window); n < 2^30.
struct OwnedWindowLabels {
    int* lds;
    unsigned cnt;
    int* G;
    __amdgpu_buffer_rsrc_t rsrc;
    unsigned oob;  // 4 n
    __device__ __forceinline__ int ld(int x) const
    {
        typedef __attribute__((address_space(3))) const int* lds_ptr;
        const unsigned i = (unsigned)x;
        const bool in = i < cnt;
        const int vl = ((lds_ptr)lds)[in ? i : 0];
        int vg = 0;
        if (__builtin_amdgcn_ballot_w64(!in) != 0)
            vg = __builtin_amdgcn_raw_buffer_load_b32(rsrc, in ? oob : i * 4u, 0, 0);
        return in ? vl : vg;
    }
    template <bool ATOMIC>
    __device__ __forceinline__ void st(int x, int z) const
    {
        if ((unsigned)x < cnt) {
            if (ATOMIC)
                atomicMin(&lds[x], z);
            else
                lds[x] = z;
        } else {
            put<ATOMIC>(G, x, z);
        }
    }
};

template <int EPT, int BLOCK, bool ATOMIC>
__device__ __forceinline__ bool run_tiles_order(const int* __restrict__ src, const int* __restrict__ dst,
                                                const int* R, int* W, long long first, long long count,
                                                long long stride, long long m, unsigned n, int h,
                                                int& rerr, int* nread = nullptr)
{
    const FlatLabels lab{R, W};
    return run_tiles_lab<EPT, BLOCK, ATOMIC>(src, dst, lab, first, count, stride, m, n, h, rerr, nread);
}

// Loop control read back from shared memory must be visibly uniform: the
// compiler cannot tell that every lane read the same word, and a loop whose
// exit looks divergent may be restructured so that some lanes of a wave go
// round a barrier again while others wait outside it.  Reading the value
// through readfirstlane makes it a scalar and the branch uniform.
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ long long uniform(long long x)
{
    const unsigned long long u = (unsigned long long)x;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

// Wait until every store this thread issued has completed, so a barrier that
// follows publishes them to the rest of the workgroup's release.
__device__ __forceinline__ void drain_stores() { __builtin_amdgcn_s_waitcnt(0); }

__device__ __forceinline__ unsigned long long ld_acquire(const unsigned long long* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int ld_acquire(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace contour
