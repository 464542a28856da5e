// contour_noalloc.hip -- contour_cc_noalloc: the single-graph persistent
// solve of contour_cc_ex without any allocation, for callers that cannot
// allocate (code under stream capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// The solve's scratch -- its control block and, when the edges are grouped,
// the grouped copy and the count tables of the grouping -- lives in one
// file-scope device array of fixed size.  Host code never passes the array's
// name to a kernel (on the host that name is only a stand-in, not a device
// address): the device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept per device.  Every
// call on a device shares that device's array, so calls that overlap on one
// device race; the control block is reset by a kernel at the start of every
// call, and the grouping tables are fully rewritten by the grouping itself.
#include <hip/hip_runtime.h>

#include <mutex>

#include "contour.h"
#include "contour_runtime.hpp"

namespace contour {

// Layout of the array: the control block in the first 256 bytes, then the
// grouping workspace (grouped src, grouped dst, count tables).
constexpr long long kNoAllocCtlInts = 256 / sizeof(int);
constexpr long long kNoAllocInts = (long long)CONTOUR_NOALLOC_SCRATCH_BYTES / sizeof(int);

static __device__ __align__(256) int scratch[kNoAllocInts];

constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current device (looked up once per
// device, with the device current).
static int scratch_address(int** out)
{
    static std::mutex mu;
    static int* addr[kMaxDevices] = {};
    int dev = 0;
    CONTOUR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return CONTOUR_ENOTSUP;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        CONTOUR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return CONTOUR_EHIP;
        addr[dev] = static_cast<int*>(p);
    }
    *out = addr[dev];
    return CONTOUR_OK;
}

}  // namespace contour

extern "C" {

int contour_cc_noalloc(const int32_t* src, const int32_t* dst, int64_t m, int32_t n, int32_t* labels_inout,
                       const contour_opts_t* opts, contour_stats_t* stats, contour_stream_t stream)
{
    if (m < 0 || n < 0) return CONTOUR_EINVAL;
    if (n > 0 && !labels_inout) return CONTOUR_EINVAL;
    if (m > 0 && (!src || !dst)) return CONTOUR_EINVAL;
    contour::Resolved r;
    int rc = contour::resolve_opts(opts, &r);
    if (rc) return rc;
    // the host-sequenced driver reads its control block through pinned host
    // memory, which would have to be allocated
    if (r.driver != CONTOUR_DRIVER_PERSISTENT) return CONTOUR_ENOTSUP;
    hipStream_t s = (hipStream_t)stream;
    int* base = nullptr;
    rc = contour::scratch_address(&base);
    if (rc) return rc;
    contour::Ctl* ctl = reinterpret_cast<contour::Ctl*>(base);
    if (n == 0) {
        // no vertices: any edge has an id outside [0, 0), reported without
        // the edges being read
        return stats ? contour::enqueue_empty_stats(ctl, stats, m > 0 ? 1 : 0, s) : CONTOUR_OK;
    }
    contour::DeviceInfo d;
    rc = contour::device_info(&d);
    if (rc) return rc;
    int* ws = nullptr;
    if (m > 0 && contour::wants_reorder(r, m, n)) {
        const long long room = contour::kNoAllocInts - contour::kNoAllocCtlInts;
        contour::Reorder ro;
        contour::solve_reorder_geometry(d, r, m, n, &ro);
        if (ro.elems > room && ro.R > 0 && r.dst_ranges == CONTOUR_DST_RANGES_AUTO) {
            // the second pass needs a second copy: without it the copy may fit
            r.dst_ranges = CONTOUR_DST_RANGES_OFF;
            contour::solve_reorder_geometry(d, r, m, n, &ro);
        }
        if (ro.elems <= room)
            ws = base + contour::kNoAllocCtlInts;
        else if (r.reorder == CONTOUR_REORDER_ON)
            return CONTOUR_ETOOBIG;
        else
            r.reorder = CONTOUR_REORDER_OFF;  // automatic grouping only where the copy fits
    }
    contour::PersistentLaunch p;
    rc = contour::prepare_persistent(d, r, src, dst, m, n, labels_inout, ctl, ws, &p);
    if (rc) return rc;
    hipEvent_t ev_begin = nullptr, ev_end = nullptr;
    contour::timing_events(&ev_begin, &ev_end);
    return contour::enqueue_persistent(p, stats, s, ev_begin, ev_end);
}

}  // extern "C"
