// contour_runtime.hpp -- host runtime shared by the single-graph and batched
// entry points: error state, device properties, per-(device, stream)
// workspaces and option resolution.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "contour.h"
#include "contour_device.hpp"

namespace contour {

// Remember a failing HIP call for contour_last_hip_error() and map it.
int hip_fail(hipError_t e);

#define CONTOUR_HIP(call)                                  \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return ::contour::hip_fail(e_); \
    } while (0)

struct DeviceInfo {
    int device = -1;
    int cus = 0;
    int wall_clock_khz = 0;
    int max_lds_per_block = 0;
    int max_threads_per_cu = 0;
};

// Properties of the current device (cached).
int device_info(DeviceInfo* out);

// Workspace bound to one (device, stream): a control block and a host-pinned
// mirror for the host-loop driver, and a grow-only scratch array.
struct Workspace {
    Ctl* ctl = nullptr;       // device
    Ctl* host_ctl = nullptr;  // host pinned
    int* scratch = nullptr;   // device, `scratch_elems` ints
    long long scratch_elems = 0;
    int* aux = nullptr;       // device, `aux_elems` ints: a second grow-only array
    long long aux_elems = 0;
};

// Look up (or create) the workspace of the current device and `stream`.
// The returned pointer stays valid for the life of the process.
int workspace_for(hipStream_t stream, Workspace** out);

// Make ws->scratch hold at least `elems` ints (may free and reallocate; the
// caller's stream is synchronised first when it grows).
int workspace_scratch(Workspace* ws, hipStream_t stream, long long elems);
// The same for ws->aux (inputs a call builds before its solve uses scratch).
int workspace_aux(Workspace* ws, hipStream_t stream, long long elems);

// Resolved options for a single solve.
struct Resolved {
    Sched sched;
    bool atomic;
    bool sync;
    int driver;
    int max_sweeps;
    bool warm;
    int block;
    int ept;
    int chunk_tiles;
    int grid;
    int reorder;
    int window;
    int dst_ranges;
    bool solo;  // a single graph on the whole GPU (batched plans clear it for their class-2 graphs)
};

// Wall-clock ticks a single solve may run before the watchdog stops it
// (CONTOUR_WATCHDOG_MS, default 60000 ms; 0 disables it).
unsigned long long watchdog_ticks(const DeviceInfo& d);

// Per-thread timing events set by contour_set_timing_events (may be null).
void timing_events(hipEvent_t* begin, hipEvent_t* end);

// One graph of a batch solved by a single workgroup (contour_batch.hip):
// its own edge and label arrays, local ids.
struct BatchJob {
    const int* src;
    const int* dst;
    int* labels;
    long long m;  // edge count
    int n;        // vertex count
    int g;        // index for stats
};

// Enqueue single-workgroup solves of `count` jobs whose table is already in
// device memory (d_jobs), on `stream`, without allocating: graphs with
// n <= lds_max keep their labels in LDS (one launch sized for the largest
// such n), the rest in global memory.  d_counters: 4 ints; d_clock: one Ctl.
// Jobs must be ordered so that the LDS ones (n <= lds_max) come first;
// n_lds of them, max_n_lds their largest n.
int enqueue_wg_jobs(const DeviceInfo& d, const Resolved& r, const BatchJob* d_jobs, int n_lds, int max_n_lds,
                    int n_global, int* d_counters, Ctl* d_clock, contour_stats_t* stats, hipStream_t stream);

// Edge reordering by source block (contour_reorder.hip), optionally followed
// by a stable second pass by destination range: the edges then come in
// (destination range, source block) order.
struct Reorder {
    int shift = 0;          // source block = src >> shift
    int K = 0;              // source blocks (at most 1024)
    int dshift = 0;         // destination range = dst >> dshift (0: no second pass)
    int R = 0;              // destination ranges (at most 64)
    long long m = 0;
    long long elems = 0;    // workspace ints needed
    int* src2 = nullptr;    // workspace: reordered edges
    int* dst2 = nullptr;
    int* src1 = nullptr;    // workspace: edges grouped by source block (second pass only)
    int* dst1 = nullptr;
    long long chunks = 0;   // 8 Ki-edge chunks of the edge list
    long long groups = 0;   // groups of 128 chunks
    int* cnt = nullptr;     // workspace: chunks x K edges per (chunk, block), then their first slots
    int* part = nullptr;    // workspace: groups x K edges per (group, block), then their first slots
    int* cnt2 = nullptr;    // the same for the second pass (R columns)
    int* part2 = nullptr;
};

// Sizes for m edges over n > 0 vertices; dshift > 0 adds the second pass by
// destination range dst >> dshift (at most 64 ranges).
void reorder_geometry(const DeviceInfo& d, long long m, int n, Reorder* r, int dshift = 0);
// Point the reorder at a workspace of at least r->elems ints.
void reorder_bind(Reorder* r, int* ws);
// Ints of that workspace besides the grouped copy (count tables).
long long reorder_table_elems(const Reorder& r);
// Point only the count tables at `tables` (reorder_table_elems ints); the
// grouped copy goes to r->src2 / r->dst2 as set by the caller.
void reorder_bind_tables(Reorder* r, int* tables);
// Enqueue the counting sort of (src, dst) into r.src2 / r.dst2.
int enqueue_reorder(const Reorder& r, const int* src, const int* dst, hipStream_t stream);
// Whether the automatic policy reorders a graph of this size.
inline bool reorder_auto(long long m, int n) { return n > (1 << 20) && m >= (1 << 20); }
// Whether a solve with these options groups its edges first.
bool wants_reorder(const Resolved& r, long long m, int n);
// The destination-range shift of a grouped solve with these options (0: no
// second pass).
int dst_range_shift(const Resolved& r, long long m, int n);
// reorder_geometry of a solve with these options (both passes as it groups).
void solve_reorder_geometry(const DeviceInfo& d, const Resolved& r, long long m, int n, Reorder* ro);

// A prepared single-graph persistent solve: everything needed to enqueue it
// without allocating (used by contour_cc_ex and by batched plans).
struct PersistentLaunch {
    void (*kernel)(SolveArgs);  // null when m == 0
    SolveArgs args;
    unsigned grid;
    int block;
    size_t lds;                 // dynamic LDS bytes (label window)
    unsigned init_blocks;
    int warm;
    int n;
    bool reorder;
    Reorder ro;
    const int* src_in;  // caller's edges (read by the reorder)
    const int* dst_in;
};

// Resolve geometry and fill *out for a solve that uses control block `ctl`.
// When the options ask for reordering, `ws` must hold reorder elems ints
// (see reorder_geometry) and the sweeps read the reordered copy.
int prepare_persistent(const DeviceInfo& d, const Resolved& r, const int* src, const int* dst,
                       long long m, int n, int* L, Ctl* ctl, int* ws, PersistentLaunch* out);

// Enqueue: reset the control block, initialise (or check) labels, run the
// persistent sweep kernel, write stats.  Optional events bracket the sweeps.
int enqueue_persistent(const PersistentLaunch& p, contour_stats_t* stats, hipStream_t stream,
                       hipEvent_t ev_begin, hipEvent_t ev_end);

// Enqueue the statistics of a solve with no vertices: status OK, or
// CONTOUR_ERANGE when range_err (there were edges, so some id lies outside
// [0, 0)).  ctl is reset first.
int enqueue_empty_stats(Ctl* ctl, contour_stats_t* stats, int range_err, hipStream_t stream);

// Validate opts and fill defaults; returns CONTOUR_OK or CONTOUR_EINVAL /
// CONTOUR_ENOTSUP.
int resolve_opts(const contour_opts_t* opts, Resolved* r);

}  // namespace contour
