// contour_runtime.cpp -- host runtime: error state, device properties,
// per-(device, stream) workspaces and option resolution.
#include "contour_runtime.hpp"

#include <cstdlib>
#include <map>
#include <mutex>
#include <utility>

namespace contour {

static thread_local int g_last_hip_error = 0;
static thread_local hipEvent_t g_ev_begin = nullptr;
static thread_local hipEvent_t g_ev_end = nullptr;

void timing_events(hipEvent_t* begin, hipEvent_t* end)
{
    *begin = g_ev_begin;
    *end = g_ev_end;
}

int hip_fail(hipError_t e)
{
    g_last_hip_error = (int)e;
    if (e == hipErrorOutOfMemory) return CONTOUR_ENOMEM;
    return CONTOUR_EHIP;
}

int device_info(DeviceInfo* out)
{
    static std::mutex mu;
    static std::map<int, DeviceInfo> cache;
    int dev = 0;
    CONTOUR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) {
        *out = it->second;
        return CONTOUR_OK;
    }
    DeviceInfo d;
    d.device = dev;
    CONTOUR_HIP(hipDeviceGetAttribute(&d.cus, hipDeviceAttributeMultiprocessorCount, dev));
    CONTOUR_HIP(hipDeviceGetAttribute(&d.max_lds_per_block,
                                      hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    CONTOUR_HIP(hipDeviceGetAttribute(&d.max_threads_per_cu,
                                      hipDeviceAttributeMaxThreadsPerMultiProcessor, dev));
    CONTOUR_HIP(hipDeviceGetAttribute(&d.wall_clock_khz, hipDeviceAttributeWallClockRate, dev));
    cache[dev] = d;
    *out = d;
    return CONTOUR_OK;
}

unsigned long long watchdog_ticks(const DeviceInfo& d)
{
    static long long ms = -1;
    if (ms < 0) {
        const char* e = getenv("CONTOUR_WATCHDOG_MS");
        ms = e ? atoll(e) : 60000;
        if (ms < 0) ms = 0;
    }
    unsigned long long khz = d.wall_clock_khz > 0 ? (unsigned long long)d.wall_clock_khz : 100000ULL;
    return (unsigned long long)ms * khz;
}

int workspace_for(hipStream_t stream, Workspace** out)
{
    static std::mutex mu;
    static std::map<std::pair<int, hipStream_t>, Workspace*> cache;
    int dev = 0;
    CONTOUR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    auto key = std::make_pair(dev, stream);
    auto it = cache.find(key);
    if (it != cache.end()) {
        *out = it->second;
        return CONTOUR_OK;
    }
    Workspace* ws = new Workspace();
    hipError_t e = hipMalloc((void**)&ws->ctl, sizeof(Ctl));
    if (e == hipSuccess) e = hipHostMalloc((void**)&ws->host_ctl, sizeof(Ctl), hipHostMallocDefault);
    if (e != hipSuccess) {
        if (ws->ctl) (void)hipFree(ws->ctl);
        delete ws;
        return hip_fail(e);
    }
    cache[key] = ws;
    *out = ws;
    return CONTOUR_OK;
}

int workspace_scratch(Workspace* ws, hipStream_t stream, long long elems)
{
    if (ws->scratch_elems >= elems) return CONTOUR_OK;
    CONTOUR_HIP(hipStreamSynchronize(stream));
    if (ws->scratch) {
        CONTOUR_HIP(hipFree(ws->scratch));
        ws->scratch = nullptr;
        ws->scratch_elems = 0;
    }
    CONTOUR_HIP(hipMalloc((void**)&ws->scratch, sizeof(int) * (size_t)elems));
    ws->scratch_elems = elems;
    return CONTOUR_OK;
}

int workspace_aux(Workspace* ws, hipStream_t stream, long long elems)
{
    if (ws->aux_elems >= elems) return CONTOUR_OK;
    CONTOUR_HIP(hipStreamSynchronize(stream));
    if (ws->aux) {
        CONTOUR_HIP(hipFree(ws->aux));
        ws->aux = nullptr;
        ws->aux_elems = 0;
    }
    CONTOUR_HIP(hipMalloc((void**)&ws->aux, sizeof(int) * (size_t)elems));
    ws->aux_elems = elems;
    return CONTOUR_OK;
}

int resolve_opts(const contour_opts_t* o, Resolved* r)
{
    contour_opts_t d;
    contour_default_opts(&d);
    if (!o) o = &d;
    int order = o->order == 0 ? 2 : o->order;
    if (!(order == CONTOUR_ORDER_FULL || (order >= 1 && order <= CONTOUR_ORDER_MAX)))
        return CONTOUR_EINVAL;
    if (o->schedule < CONTOUR_SCHED_FIXED || o->schedule > CONTOUR_SCHED_1M1M) return CONTOUR_EINVAL;
    if (o->k1 < 0 || o->max_sweeps < 0 || o->warm_start < 0 || o->warm_start > 1)
        return CONTOUR_EINVAL;
    if (o->write_mode != CONTOUR_WRITE_PLAIN && o->write_mode != CONTOUR_WRITE_ATOMIC)
        return CONTOUR_EINVAL;
    if (o->update != CONTOUR_UPDATE_ASYNC && o->update != CONTOUR_UPDATE_SYNC) return CONTOUR_EINVAL;
    if (o->driver != CONTOUR_DRIVER_PERSISTENT && o->driver != CONTOUR_DRIVER_HOSTLOOP)
        return CONTOUR_EINVAL;
    if (o->block != 0 && o->block != 256 && o->block != 512 && o->block != 1024) return CONTOUR_EINVAL;
    if (o->edges_per_thread != 0 && o->edges_per_thread != 1 && o->edges_per_thread != 2 &&
        o->edges_per_thread != 4 && o->edges_per_thread != 8)
        return CONTOUR_EINVAL;
    if (o->chunk_tiles < 0 || o->grid < 0) return CONTOUR_EINVAL;
    if (o->reorder < CONTOUR_REORDER_AUTO || o->reorder > CONTOUR_REORDER_ON) return CONTOUR_EINVAL;
    if (o->window != 0 && o->window < 1024) return CONTOUR_EINVAL;
    if (!(o->dst_ranges == CONTOUR_DST_RANGES_AUTO || o->dst_ranges == CONTOUR_DST_RANGES_OFF ||
          o->dst_ranges == CONTOUR_DST_RANGES_ON || (o->dst_ranges >= 16 && o->dst_ranges <= 30)))
        return CONTOUR_EINVAL;
    // Algorithm 1 applies its conditional assignments to L_u with the
    // compare-and-swap loop of Eq. (cas); the synchronous update is only
    // offered that way, and sequenced from the host.
    if (o->update == CONTOUR_UPDATE_SYNC &&
        (o->write_mode != CONTOUR_WRITE_ATOMIC || o->driver != CONTOUR_DRIVER_HOSTLOOP))
        return CONTOUR_ENOTSUP;
    r->sched.order = order;
    r->sched.kind = o->schedule;
    r->sched.k1 = o->k1 == 0 ? 2 : o->k1;
    r->atomic = o->write_mode == CONTOUR_WRITE_ATOMIC;
    r->sync = o->update == CONTOUR_UPDATE_SYNC;
    r->driver = o->driver;
    r->max_sweeps = o->max_sweeps;
    r->warm = o->warm_start == 1;
    r->block = o->block;
    r->ept = o->edges_per_thread;
    r->chunk_tiles = o->chunk_tiles;
    r->grid = o->grid;
    r->reorder = o->reorder;
    r->window = o->window;
    r->dst_ranges = o->dst_ranges;
    r->solo = true;
    return CONTOUR_OK;
}

}  // namespace contour

extern "C" {

void contour_default_opts(contour_opts_t* opts)
{
    if (!opts) return;
    opts->order = 0;  // the default order: 2 for a solve, the tuned order in a batched plan
    opts->schedule = CONTOUR_SCHED_FIXED;
    opts->k1 = 2;
    opts->write_mode = CONTOUR_WRITE_PLAIN;
    opts->update = CONTOUR_UPDATE_ASYNC;
    opts->driver = CONTOUR_DRIVER_PERSISTENT;
    opts->max_sweeps = 0;
    opts->warm_start = 0;
    opts->block = 0;
    opts->edges_per_thread = 0;
    opts->chunk_tiles = 0;
    opts->grid = 0;
    opts->reorder = CONTOUR_REORDER_AUTO;
    opts->window = 0;
    opts->dst_ranges = CONTOUR_DST_RANGES_AUTO;
}

const char* contour_status_string(int s)
{
    switch (s) {
    case CONTOUR_OK: return "ok";
    case CONTOUR_EINVAL: return "invalid argument";
    case CONTOUR_ERANGE: return "edge id outside [0, n)";
    case CONTOUR_ENOMEM: return "device allocation failed";
    case CONTOUR_EHIP: return "HIP runtime error";
    case CONTOUR_ENOCONV: return "sweep limit reached before convergence";
    case CONTOUR_ENOTSUP: return "option combination not supported";
    case CONTOUR_ETOOBIG: return "input needs more than the fixed no-allocation scratch";
    default: return "unknown status";
    }
}

int contour_last_hip_error(void) { return contour::g_last_hip_error; }

void contour_set_timing_events(void* begin, void* end)
{
    contour::g_ev_begin = (hipEvent_t)begin;
    contour::g_ev_end = (hipEvent_t)end;
}

const char* contour_version(void) { return "contour-mi355x 0.1 (gfx950)"; }

}  // extern "C"
