// contour_serve.cpp -- the serving loop of contour_serve.h.
//
// One engine thread owns the device work.  Each pass of its loop
//   1. retires lanes whose completion event has fired (labels and stats are
//      back in host memory): results are timestamped and their device
//      memory returns to the pool;
//   2. refills every idle lane from the queue, in arrival order: either a
//      micro-batch of small requests (one workgroup per graph, one launch)
//      or one large request (persistent multi-workgroup solve), admitting
//      each request only when its device footprint fits the HBM budget;
//   3. when nothing changed: yields while lanes are in flight (their
//      completion is found by polling events), and waits for the next
//      submission when nothing is in flight.
// A lane is a stream plus the small tables its launches need, allocated once
// at creation, so serving allocates device memory only through the request
// pool (power-of-two size classes, reused, counted against the budget).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "contour.h"
#include "contour_runtime.hpp"
#include "contour_serve.h"

namespace contour {
namespace {

int64_t now_ns()
{
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t round_pow2(size_t x)
{
    size_t p = 256;
    while (p < x) p <<= 1;
    return p;
}

struct Request {
    int64_t id = 0;
    const int* h_src = nullptr;
    const int* h_dst = nullptr;
    int* h_labels = nullptr;
    int64_t m = 0;
    int n = 0;
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    int status = CONTOUR_OK;
    int sweeps = 0;
    size_t bytes = 0;  // pool block size (0: none)
    void* block = nullptr;
    int* d_src = nullptr;
    int* d_dst = nullptr;
    int* d_lab = nullptr;
};

struct Lane {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    bool big = false;
    std::vector<Request*> reqs;
    BatchJob* h_jobs = nullptr;  // pinned, batch_max
    BatchJob* d_jobs = nullptr;
    contour_stats_t* h_stats = nullptr;  // pinned, batch_max
    contour_stats_t* d_stats = nullptr;
    int* d_counters = nullptr;
    Ctl* d_clock = nullptr;
    Ctl* d_ctl = nullptr;        // large requests
    int* d_ws = nullptr;         // large requests: reorder workspace
    long long ws_elems = 0;
};

}  // namespace
}  // namespace contour

struct contour_server {
    contour_server_config_t cfg;
    contour::Resolved r;
    contour::DeviceInfo dev;
    int lds_max = 0;
    std::vector<contour::Lane> lanes;
    std::thread engine;
    std::mutex mu;
    std::condition_variable cv_done;
    std::condition_variable cv_work;  // the engine waits here when it has nothing in flight
    std::deque<contour::Request*> pending;  // submitted, not yet admitted
    std::deque<contour::Request*> finished;
    int64_t next_id = 1;
    int64_t submitted = 0, completed = 0;
    bool stop = false;
    std::atomic<int> fatal{0};
    // pool
    std::map<size_t, std::vector<void*>> free_blocks;
    size_t in_use = 0;     // bytes of blocks held by admitted requests and lane workspaces
    size_t cached = 0;     // bytes of free blocks kept for reuse
};

namespace contour {
namespace {

void* pool_get(contour_server* s, size_t bytes)
{
    auto it = s->free_blocks.find(bytes);
    if (it != s->free_blocks.end() && !it->second.empty()) {
        void* p = it->second.back();
        it->second.pop_back();
        s->cached -= bytes;
        s->in_use += bytes;
        return p;
    }
    // release cached blocks of other sizes if the new block would not fit
    size_t budget = (size_t)s->cfg.hbm_budget_bytes;
    for (auto fit = s->free_blocks.begin(); s->in_use + s->cached + bytes > budget && fit != s->free_blocks.end();
         ++fit) {
        while (!fit->second.empty() && s->in_use + s->cached + bytes > budget) {
            (void)hipFree(fit->second.back());
            fit->second.pop_back();
            s->cached -= fit->first;
        }
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    s->in_use += bytes;
    return p;
}

void pool_put(contour_server* s, void* p, size_t bytes)
{
    s->in_use -= bytes;
    s->cached += bytes;
    s->free_blocks[bytes].push_back(p);
}

size_t footprint(int64_t m, int n)
{
    const size_t e = (size_t)m * sizeof(int), l = (size_t)n * sizeof(int);
    return round_pow2(2 * ((e + 255) & ~(size_t)255) + ((l + 255) & ~(size_t)255) + 256);
}

// Try to give r its device memory within the budget.
bool admit(contour_server* s, Request* r)
{
    const size_t bytes = footprint(r->m, r->n);
    if (s->in_use + bytes > (size_t)s->cfg.hbm_budget_bytes) return false;
    void* p = pool_get(s, bytes);
    if (!p) return false;
    r->block = p;
    r->bytes = bytes;
    char* c = (char*)p;
    const size_t e = ((size_t)r->m * sizeof(int) + 255) & ~(size_t)255;
    r->d_src = (int*)c;
    r->d_dst = (int*)(c + e);
    r->d_lab = (int*)(c + 2 * e);
    r->t_admit = now_ns();
    return true;
}

void release(contour_server* s, Request* r)
{
    if (r->block) pool_put(s, r->block, r->bytes);
    r->block = nullptr;
    r->bytes = 0;
}

int launch_small(contour_server* s, Lane& L)
{
    const int cnt = (int)L.reqs.size();
    for (Request* r : L.reqs) {
        if (r->m > 0) {
            CONTOUR_HIP(hipMemcpyAsync(r->d_src, r->h_src, sizeof(int) * (size_t)r->m, hipMemcpyHostToDevice, L.stream));
            CONTOUR_HIP(hipMemcpyAsync(r->d_dst, r->h_dst, sizeof(int) * (size_t)r->m, hipMemcpyHostToDevice, L.stream));
        }
    }
    // LDS-resident graphs first, then the rest
    int n_lds = 0, max_n = 0, k = 0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i < cnt; ++i) {
            Request* r = L.reqs[i];
            const bool lds = r->n <= s->lds_max;
            if ((pass == 0) != lds) continue;
            BatchJob& j = L.h_jobs[k++];
            j.src = r->d_src;
            j.dst = r->d_dst;
            j.labels = r->d_lab;
            j.m = r->m;
            j.n = r->n;
            j.g = i;
            if (lds) {
                ++n_lds;
                max_n = std::max(max_n, r->n);
            }
        }
    }
    CONTOUR_HIP(hipMemcpyAsync(L.d_jobs, L.h_jobs, sizeof(BatchJob) * (size_t)cnt, hipMemcpyHostToDevice, L.stream));
    int rc = enqueue_wg_jobs(s->dev, s->r, L.d_jobs, n_lds, max_n, cnt - n_lds, L.d_counters, L.d_clock, L.d_stats,
                             L.stream);
    if (rc) return rc;
    for (Request* r : L.reqs)
        CONTOUR_HIP(hipMemcpyAsync(r->h_labels, r->d_lab, sizeof(int) * (size_t)r->n, hipMemcpyDeviceToHost, L.stream));
    CONTOUR_HIP(hipMemcpyAsync(L.h_stats, L.d_stats, sizeof(contour_stats_t) * (size_t)cnt, hipMemcpyDeviceToHost,
                               L.stream));
    CONTOUR_HIP(hipEventRecord(L.done, L.stream));
    return CONTOUR_OK;
}

int launch_big(contour_server* s, Lane& L)
{
    Request* r = L.reqs[0];
    CONTOUR_HIP(hipMemcpyAsync(r->d_src, r->h_src, sizeof(int) * (size_t)r->m, hipMemcpyHostToDevice, L.stream));
    CONTOUR_HIP(hipMemcpyAsync(r->d_dst, r->h_dst, sizeof(int) * (size_t)r->m, hipMemcpyHostToDevice, L.stream));
    PersistentLaunch p;
    int rc = prepare_persistent(s->dev, s->r, r->d_src, r->d_dst, r->m, r->n, r->d_lab, L.d_ctl, L.d_ws, &p);
    if (rc) return rc;
    rc = enqueue_persistent(p, L.d_stats, L.stream, nullptr, nullptr);
    if (rc) return rc;
    CONTOUR_HIP(hipMemcpyAsync(r->h_labels, r->d_lab, sizeof(int) * (size_t)r->n, hipMemcpyDeviceToHost, L.stream));
    CONTOUR_HIP(hipMemcpyAsync(L.h_stats, L.d_stats, sizeof(contour_stats_t), hipMemcpyDeviceToHost, L.stream));
    CONTOUR_HIP(hipEventRecord(L.done, L.stream));
    return CONTOUR_OK;
}

// Reorder workspace of a lane for a large request (kept for reuse).
bool ensure_workspace(contour_server* s, Lane& L, const Request* r)
{
    Resolved rr = s->r;
    long long need = 0;
    const bool reorder = rr.reorder == CONTOUR_REORDER_ON ||
                         (rr.reorder == CONTOUR_REORDER_AUTO && reorder_auto(r->m, r->n));
    if (reorder && r->m < 0x7fffffffLL) {
        Reorder ro;
        solve_reorder_geometry(s->dev, rr, r->m, r->n, &ro);
        need = ro.elems;
    }
    if (need <= L.ws_elems) return true;
    const size_t old_bytes = L.d_ws ? round_pow2(sizeof(int) * (size_t)L.ws_elems) : 0;
    const size_t bytes = round_pow2(sizeof(int) * (size_t)need);
    if (s->in_use - old_bytes + bytes > (size_t)s->cfg.hbm_budget_bytes) return false;
    if (L.d_ws) {
        pool_put(s, L.d_ws, old_bytes);
        L.d_ws = nullptr;
        L.ws_elems = 0;
    }
    void* p = pool_get(s, bytes);
    if (!p) return false;
    L.d_ws = (int*)p;
    L.ws_elems = (long long)(bytes / sizeof(int));
    return true;
}

void finish(contour_server* s, Request* r, int status, int sweeps)
{
    r->status = status;
    r->sweeps = sweeps;
    r->t_done = now_ns();
    release(s, r);
    std::lock_guard<std::mutex> lock(s->mu);
    s->finished.push_back(r);
    ++s->completed;
    s->cv_done.notify_all();
}

void engine_loop(contour_server* s)
{
    (void)hipSetDevice(s->dev.device);
    for (;;) {
        bool progress = false;
        // 1. retire finished lanes
        for (Lane& L : s->lanes) {
            if (!L.busy) continue;
            const hipError_t q = hipEventQuery(L.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) s->fatal = (int)q;
            for (size_t i = 0; i < L.reqs.size(); ++i) {
                const contour_stats_t& st = L.h_stats[i];
                finish(s, L.reqs[i], q == hipSuccess ? st.status : CONTOUR_EHIP, st.sweeps_executed);
            }
            L.reqs.clear();
            L.busy = false;
            progress = true;
        }
        // 2. refill idle lanes in arrival order
        for (Lane& L : s->lanes) {
            if (L.busy) continue;
            std::vector<Request*> take, answer;
            bool big = false, blocked = false;
            {
                std::lock_guard<std::mutex> lock(s->mu);
                while (!s->pending.empty() && (int)take.size() < s->cfg.batch_max) {
                    Request* r = s->pending.front();
                    if (r->n == 0 || footprint(r->m, r->n) > (size_t)s->cfg.hbm_budget_bytes) {
                        // nothing to solve, or can never fit: answer at once
                        s->pending.pop_front();
                        r->status = r->n == 0 ? (r->m > 0 ? CONTOUR_ERANGE : CONTOUR_OK) : CONTOUR_ENOMEM;
                        r->t_admit = now_ns();
                        answer.push_back(r);
                        continue;
                    }
                    const bool is_big = r->m > s->cfg.small_edges;
                    if (is_big && !take.empty()) break;  // launch the small ones first
                    if ((is_big && !ensure_workspace(s, L, r)) || !admit(s, r)) {
                        blocked = take.empty();          // wait for memory to free up
                        break;
                    }
                    s->pending.pop_front();
                    take.push_back(r);
                    if (is_big) {
                        big = true;
                        break;
                    }
                }
            }
            for (Request* r : answer) {
                finish(s, r, r->status, 0);
                progress = true;
            }
            if (blocked) {
                // Nothing could be admitted.  With no lane in flight the only
                // memory held is cached lane workspaces: return them so the
                // next pass can use the whole budget.
                bool any_busy = false;
                for (const Lane& M : s->lanes) any_busy |= M.busy;
                if (!any_busy) {
                    bool freed = false;
                    for (Lane& M : s->lanes) {
                        if (M.d_ws) {
                            pool_put(s, M.d_ws, round_pow2(sizeof(int) * (size_t)M.ws_elems));
                            M.d_ws = nullptr;
                            M.ws_elems = 0;
                            freed = true;
                        }
                    }
                    progress |= freed;
                    if (!freed) {
                        // the queue head cannot be admitted even on an idle
                        // device: fail it rather than wait forever
                        Request* r = nullptr;
                        {
                            std::lock_guard<std::mutex> lock(s->mu);
                            if (!s->pending.empty()) {
                                r = s->pending.front();
                                s->pending.pop_front();
                            }
                        }
                        if (r) {
                            r->t_admit = now_ns();
                            finish(s, r, CONTOUR_ENOMEM, 0);
                            progress = true;
                        }
                    }
                }
                break;
            }
            if (take.empty()) continue;
            L.reqs = take;
            L.big = big;
            const int rc = big ? launch_big(s, L) : launch_small(s, L);
            if (rc != CONTOUR_OK) {
                for (Request* r : L.reqs) finish(s, r, rc, 0);
                L.reqs.clear();
                continue;
            }
            L.busy = true;
            progress = true;
        }
        // 3. stop or wait
        bool any_busy = false;
        for (const Lane& L : s->lanes) any_busy |= L.busy;
        {
            std::unique_lock<std::mutex> lock(s->mu);
            const bool idle = s->pending.empty();
            if (s->stop && idle && !any_busy) break;
            if (!progress && !any_busy) {
                // nothing in flight: sleep until a submission or stop (at
                // most 1 ms, so a request waiting for memory is retried)
                const auto seen = s->submitted;
                s->cv_work.wait_for(lock, std::chrono::milliseconds(1),
                                    [&] { return s->stop || s->submitted != seen; });
                continue;
            }
        }
        // lanes in flight: poll their events again soon, without sleeping
        // (a sleep of the engine thread adds tens of microseconds to every
        // request's latency)
        if (!progress) std::this_thread::yield();
    }
}

void destroy_lanes(contour_server* s)
{
    for (Lane& L : s->lanes) {
        if (L.stream) (void)hipStreamSynchronize(L.stream);
        if (L.done) (void)hipEventDestroy(L.done);
        if (L.stream) (void)hipStreamDestroy(L.stream);
        if (L.h_jobs) (void)hipHostFree(L.h_jobs);
        if (L.h_stats) (void)hipHostFree(L.h_stats);
        if (L.d_jobs) (void)hipFree(L.d_jobs);
        if (L.d_stats) (void)hipFree(L.d_stats);
        if (L.d_counters) (void)hipFree(L.d_counters);
        if (L.d_clock) (void)hipFree(L.d_clock);
        if (L.d_ctl) (void)hipFree(L.d_ctl);
        if (L.d_ws) (void)hipFree(L.d_ws);
    }
    s->lanes.clear();
    for (auto& kv : s->free_blocks)
        for (void* p : kv.second) (void)hipFree(p);
    s->free_blocks.clear();
}

}  // namespace
}  // namespace contour

extern "C" {

void contour_server_default_config(contour_server_config_t* c)
{
    if (!c) return;
    c->hbm_budget_bytes = 0;
    c->lanes = 4;
    c->batch_max = 512;
    c->small_edges = 1 << 20;
    contour_default_opts(&c->opts);
}

int64_t contour_server_now_ns(void) { return contour::now_ns(); }

int contour_server_create(const contour_server_config_t* cfg_in, contour_server_t* out)
{
    using namespace contour;
    if (!out) return CONTOUR_EINVAL;
    *out = nullptr;
    contour_server_config_t cfg;
    contour_server_default_config(&cfg);
    if (cfg_in) cfg = *cfg_in;
    if (cfg.lanes == 0) cfg.lanes = 4;
    if (cfg.batch_max == 0) cfg.batch_max = 512;
    if (cfg.small_edges == 0) cfg.small_edges = 1 << 20;
    if (cfg.lanes < 1 || cfg.lanes > 64 || cfg.batch_max < 1 || cfg.batch_max > 65536 || cfg.small_edges < 0 ||
        cfg.hbm_budget_bytes < 0)
        return CONTOUR_EINVAL;
    Resolved r;
    int rc = resolve_opts(&cfg.opts, &r);
    if (rc) return rc;
    if (r.sync || r.driver != CONTOUR_DRIVER_PERSISTENT || r.warm) return CONTOUR_ENOTSUP;
    contour_server* s = new (std::nothrow) contour_server();
    if (!s) return CONTOUR_ENOMEM;
    s->r = r;
    rc = device_info(&s->dev);
    if (rc) {
        delete s;
        return rc;
    }
    s->lds_max = std::min(16384, (s->dev.max_lds_per_block - 1024) / 4);
    if (cfg.hbm_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            delete s;
            return hip_fail(hipGetLastError());
        }
        cfg.hbm_budget_bytes = (int64_t)(free_b / 2);
    }
    s->cfg = cfg;
    s->lanes.resize(cfg.lanes);
    hipError_t e = hipSuccess;
    for (Lane& L : s->lanes) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&L.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void**)&L.h_jobs, sizeof(BatchJob) * cfg.batch_max, hipHostMallocDefault);
        if (e == hipSuccess)
            e = hipHostMalloc((void**)&L.h_stats, sizeof(contour_stats_t) * cfg.batch_max, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void**)&L.d_jobs, sizeof(BatchJob) * cfg.batch_max);
        if (e == hipSuccess) e = hipMalloc((void**)&L.d_stats, sizeof(contour_stats_t) * cfg.batch_max);
        if (e == hipSuccess) e = hipMalloc((void**)&L.d_counters, 4 * sizeof(int));
        if (e == hipSuccess) e = hipMalloc((void**)&L.d_clock, sizeof(Ctl));
        if (e == hipSuccess) e = hipMalloc((void**)&L.d_ctl, sizeof(Ctl));
    }
    if (e != hipSuccess) {
        destroy_lanes(s);
        delete s;
        return hip_fail(e);
    }
    s->engine = std::thread(engine_loop, s);
    *out = s;
    return CONTOUR_OK;
}

int contour_server_submit(contour_server_t s, const int32_t* h_src, const int32_t* h_dst, int64_t m, int32_t n,
                          int32_t* h_labels, int64_t* id_out)
{
    if (!s || m < 0 || n < 0 || (m > 0 && (!h_src || !h_dst)) || (n > 0 && !h_labels)) return CONTOUR_EINVAL;
    contour::Request* r = new (std::nothrow) contour::Request();
    if (!r) return CONTOUR_ENOMEM;
    r->h_src = h_src;
    r->h_dst = h_dst;
    r->h_labels = h_labels;
    r->m = m;
    r->n = n;
    r->t_submit = contour::now_ns();
    std::lock_guard<std::mutex> lock(s->mu);
    if (s->stop) {
        delete r;
        return CONTOUR_EINVAL;
    }
    r->id = s->next_id++;
    ++s->submitted;
    s->pending.push_back(r);
    if (id_out) *id_out = r->id;
    s->cv_work.notify_one();
    return CONTOUR_OK;
}

int contour_server_poll(contour_server_t s, contour_request_result_t* out, int32_t max, int32_t wait_us,
                        int32_t* count)
{
    if (!s || !count || max < 0 || (max > 0 && !out)) return CONTOUR_EINVAL;
    std::unique_lock<std::mutex> lock(s->mu);
    if (s->finished.empty() && wait_us > 0)
        s->cv_done.wait_for(lock, std::chrono::microseconds(wait_us), [&] { return !s->finished.empty(); });
    int k = 0;
    while (k < max && !s->finished.empty()) {
        contour::Request* r = s->finished.front();
        s->finished.pop_front();
        out[k].id = r->id;
        out[k].status = r->status;
        out[k].sweeps_executed = r->sweeps;
        out[k].t_submit_ns = r->t_submit;
        out[k].t_admit_ns = r->t_admit;
        out[k].t_done_ns = r->t_done;
        delete r;
        ++k;
    }
    *count = k;
    return CONTOUR_OK;
}

int contour_server_drain(contour_server_t s)
{
    if (!s) return CONTOUR_EINVAL;
    std::unique_lock<std::mutex> lock(s->mu);
    const int64_t target = s->submitted;
    s->cv_done.wait(lock, [&] { return s->completed >= target || s->fatal.load() != 0; });
    return s->fatal.load() ? CONTOUR_EHIP : CONTOUR_OK;
}

int contour_server_destroy(contour_server_t s)
{
    if (!s) return CONTOUR_OK;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->engine.joinable()) s->engine.join();
    for (contour::Request* r : s->finished) delete r;
    s->finished.clear();
    contour::destroy_lanes(s);
    delete s;
    return CONTOUR_OK;
}

}  // extern "C"
