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
};

// Look up (or create) the workspace of the current device and `stream`.
// The returned pointer stays valid for the life of the process.
int workspace_for(hipStream_t stream, Workspace** out);

// Make ws->scratch hold at least `elems` ints (may free and reallocate; the
// caller's stream is synchronised first when it grows).
int workspace_scratch(Workspace* ws, hipStream_t stream, long long elems);

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
};

// Wall-clock ticks a single solve may run before the watchdog stops it
// (CONTOUR_WATCHDOG_MS, default 60000 ms; 0 disables it).
unsigned long long watchdog_ticks(const DeviceInfo& d);

// Per-thread timing events set by contour_set_timing_events (may be null).
void timing_events(hipEvent_t* begin, hipEvent_t* end);

// A prepared single-graph persistent solve: everything needed to enqueue it
// without allocating (used by contour_cc_ex and by batched plans).
struct PersistentLaunch {
    void (*kernel)(SolveArgs);  // null when m == 0
    SolveArgs args;
    unsigned grid;
    int block;
    unsigned init_blocks;
    int warm;
    int n;
};

// Resolve geometry and fill *out for a solve that uses control block `ctl`.
int prepare_persistent(const DeviceInfo& d, const Resolved& r, const int* src, const int* dst,
                       long long m, int n, int* L, Ctl* ctl, PersistentLaunch* out);

// Enqueue: reset the control block, initialise (or check) labels, run the
// persistent sweep kernel, write stats.  Optional events bracket the sweeps.
int enqueue_persistent(const PersistentLaunch& p, contour_stats_t* stats, hipStream_t stream,
                       hipEvent_t ev_begin, hipEvent_t ev_end);

// Validate opts and fill defaults; returns CONTOUR_OK or CONTOUR_EINVAL /
// CONTOUR_ENOTSUP.
int resolve_opts(const contour_opts_t* opts, Resolved* r);

}  // namespace contour
