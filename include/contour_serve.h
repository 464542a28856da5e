/*
 * contour_serve.h -- a serving loop for connectivity requests on one MI355X.
 *
 * Requests (an undirected graph each: host int32 edge arrays and a vertex
 * count) arrive at any time.  Each result is exactly what contour_cc would
 * return for that graph alone: labels[v] = minimum vertex id of v's
 * component (Section II-A of the paper).  The server adds the systems side:
 *
 *   admission   a request is admitted when its device footprint (edges,
 *               labels, and for large graphs the solve workspace) fits in
 *               the HBM budget next to the requests already on the device;
 *               requests are admitted in arrival order;
 *   batching    admitted small requests (m <= small_edges) are launched
 *               together, one workgroup per graph, in a single launch per
 *               micro-batch; large requests get a persistent multi-workgroup
 *               solve of their own;
 *   overlap     several lanes (device streams) run at once: while one
 *               micro-batch or large request is on the GPU, the requests
 *               that arrived meanwhile are copied and launched on another
 *               lane, and finished lanes are refilled immediately
 *               (continuous batching);
 *   reporting   every request records submit, admit and completion times on
 *               the server's clock, for p50 / p99 latency.
 *
 * Threading: one engine thread per server issues all HIP calls on the
 * device that was current at creation.  contour_server_submit and
 * contour_server_poll may be called from any thread.
 *
 * Ownership: the caller keeps a request's h_src, h_dst and h_labels valid
 * and unmodified from submit until the request is reported done.  Host
 * buffers allocated with hipHostMalloc (pinned) make the copies
 * asynchronous; pageable buffers work but copy synchronously.
 */
#ifndef CONTOUR_SERVE_H
#define CONTOUR_SERVE_H

#include <stdint.h>

#include "contour.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct contour_server* contour_server_t;

typedef struct {
    int64_t hbm_budget_bytes; /* device bytes for admitted requests; 0: half the free HBM at creation */
    int32_t lanes;            /* device streams in flight at once, 1..64; 0: 4 */
    int32_t batch_max;        /* most small requests per micro-batch, 1..65536; 0: 512 */
    int64_t small_edges;      /* requests with m <= small_edges are micro-batched; 0: 2^20 */
    contour_opts_t opts;      /* solve options for every request (defaults: contour_default_opts) */
} contour_server_config_t;

typedef struct {
    int64_t id;              /* as returned by contour_server_submit */
    int32_t status;          /* contour_status_t of the solve (ENOMEM: larger than the budget) */
    int32_t sweeps_executed; /* sweeps of the request's solve */
    int64_t t_submit_ns;     /* contour_server_now_ns() at submit */
    int64_t t_admit_ns;      /* when its device memory was granted and its copy enqueued */
    int64_t t_done_ns;       /* when the engine saw its labels back in host memory */
} contour_request_result_t;

/* Fill *cfg with the defaults. */
void contour_server_default_config(contour_server_config_t* cfg);

/* Start a server on the current device.  Returns CONTOUR_OK, CONTOUR_EINVAL
 * (bad config), CONTOUR_ENOMEM or CONTOUR_EHIP. */
int contour_server_create(const contour_server_config_t* cfg, contour_server_t* out);

/* Queue one request: h_src, h_dst host int32[m] (ids in [0, n)), h_labels
 * host int32[n] written when the request is done.  *id_out receives the
 * request id.  Returns CONTOUR_OK or CONTOUR_EINVAL (bad sizes, NULL
 * arrays, or the server is shutting down). */
int contour_server_submit(contour_server_t s, const int32_t* h_src, const int32_t* h_dst, int64_t m, int32_t n,
                          int32_t* h_labels, int64_t* id_out);

/* Take up to max finished requests (oldest first) into out[]; waits up to
 * wait_us microseconds for at least one when none is ready (0: no wait).
 * *count receives the number taken. */
int contour_server_poll(contour_server_t s, contour_request_result_t* out, int32_t max, int32_t wait_us,
                        int32_t* count);

/* Block until every request submitted so far is done (results stay
 * available to contour_server_poll). */
int contour_server_drain(contour_server_t s);

/* Stop the engine after the queued requests finish, and free everything. */
int contour_server_destroy(contour_server_t s);

/* The server's clock: steady nanoseconds. */
int64_t contour_server_now_ns(void);

#ifdef __cplusplus
}
#endif

#endif /* CONTOUR_SERVE_H */
