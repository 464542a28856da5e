/*
 * contour.h -- C ABI of libcontour, exact connected components on one
 * MI355X (gfx950) by the Contour minimum-mapping algorithm
 * (Du, Alvarado Rodriguez, Li, Dindoost, Bader, "Contour Algorithm for
 * Connectivity", arXiv 2311.02811).
 *
 * What every entry point computes (Section II-A, Theorem "Graph Convergence"):
 * for an undirected graph with vertex ids 0..n-1 and an edge list, the label
 * of vertex v is the minimum vertex id of v's connected component.  The
 * result is unique, so it is the same bit for bit for every operator order,
 * write mode, schedule, launch geometry and edge order.
 *
 * How: labels start at L[i] = i (Algorithm 1, initialisation).  Each sweep
 * applies the h-order minimum-mapping operator MM^h (Definition 3) to every
 * edge <w, v>: z = min(L^h[w], L^h[v]) is written into L[x] for every x on
 * the chains w, L[w], ..., L^{h-1}[w] and v, ..., L^{h-1}[v] whose value
 * exceeds z (the conditional assignment of Definition 1).  By default the
 * array is updated in place (asynchronous update, Section III-B-1) with plain
 * stores (no atomics, Section III-B-3), and a sweep in which no edge finds
 * anything to change ends the run (early convergence check, Section III-B-2,
 * evaluated on the values each edge read before its own writes).
 *
 * Conventions shared by every entry point
 *   * Arrays are device pointers owned by the caller unless stated.  Edge
 *     arrays are int32 structure-of-arrays src[m], dst[m]; each undirected
 *     edge appears once in either orientation; self-loops and duplicates are
 *     allowed.  Label arrays must not alias the edge arrays.
 *   * Calls are stream ordered: they enqueue work on `stream` (a hipStream_t,
 *     NULL for the null stream) and return before it completes, except where
 *     a driver mode says it blocks.  Results are valid once the stream has
 *     completed the enqueued work.
 *   * The library keeps a workspace per (device, stream): a control block and
 *     a grow-only scratch array.  The first call on a stream, and a call that
 *     needs more scratch than the stream holds, allocate it (and synchronise
 *     the stream before growing it).  contour_reserve does that up front;
 *     after it, calls within the reserved sizes only enqueue kernels (no
 *     allocation, no synchronisation, no memset), so they can be captured into
 *     a hipGraph.  contour_cc_noalloc never allocates at all.
 *   * Argument errors (NULL with a non-zero size, negative sizes, bad
 *     options) are returned synchronously and nothing is enqueued.
 *   * Data errors are reported through contour_stats_t.status after the
 *     stream completes: an edge with an id outside [0, n) is skipped, never
 *     dereferenced, and status becomes CONTOUR_ERANGE (labels are then the
 *     labels of the graph without those edges); running out of sweeps gives
 *     CONTOUR_ENOCONV with a valid partial state that a warm start resumes.
 *   * HIP runtime failures return CONTOUR_EHIP; contour_last_hip_error()
 *     then gives the hipError_t of the calling thread's last failure.
 *   * The library owns a small per-(device, stream) workspace (control
 *     words); calls on different streams may run concurrently, calls on the
 *     same stream are serialised by the stream.
 */
#ifndef CONTOUR_H
#define CONTOUR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void* contour_stream_t; /* a hipStream_t */

typedef enum {
    CONTOUR_OK = 0,
    CONTOUR_EINVAL = 1,  /* bad argument or option */
    CONTOUR_ERANGE = 2,  /* an edge id outside [0, n) (reported in stats) */
    CONTOUR_ENOMEM = 3,  /* device allocation of the workspace failed */
    CONTOUR_EHIP = 4,    /* a HIP runtime call failed */
    CONTOUR_ENOCONV = 5, /* max_sweeps reached before convergence (stats) */
    CONTOUR_ENOTSUP = 6, /* option combination not supported */
    CONTOUR_ETOOBIG = 7  /* the input needs more scratch than contour_cc_noalloc's fixed array */
} contour_status_t;

/* Operator order h of MM^h (Definition 3).  1, 2 (default), 3, ... up to
 * CONTOUR_ORDER_MAX are exact orders; CONTOUR_ORDER_FULL follows each chain
 * to its root (L[x] = x) and writes z to every vertex on it, root included.
 * Because every chain strictly decreases until its root, an order larger
 * than the longest chain acts exactly like CONTOUR_ORDER_FULL. */
#define CONTOUR_ORDER_FULL (-1)
#define CONTOUR_ORDER_MAX 1024

/* Operator schedules of Section III-B-4. */
#define CONTOUR_SCHED_FIXED 0 /* `order` in every sweep (C-1, C-2, C-m) */
#define CONTOUR_SCHED_11MM 1  /* order 1 for the first k1 sweeps, then `order` (C-11mm) */
#define CONTOUR_SCHED_1M1M 2  /* order 1 and `order` alternately, from 1 (C-1m1m) */

/* Write rule of the conditional assignment. */
/* CONTOUR_WRITE_PLAIN: if (read > z) L[x] = z, a benign race (Section III-B-3),
 * in memory that one workgroup owns: LDS label windows and the labels of
 * one-workgroup batched graphs.  Label stores that workgroups on different
 * XCDs race on go to global memory as written-through stores or atomic
 * minima in either mode, on every driver: the XCDs' L2 caches are not
 * coherent for cached stores within a kernel, and plain global stores also
 * gave a wrong result once on the host-loop driver.  The labels are the
 * same either way and the early convergence check stays sound. */
#define CONTOUR_WRITE_PLAIN 0
#define CONTOUR_WRITE_ATOMIC 1 /* if (read > z) atomic_min(&L[x], z);  Eq. (cas) */

/* Update rule. */
#define CONTOUR_UPDATE_ASYNC 0 /* one array updated in place (Section III-B-1) */
#define CONTOUR_UPDATE_SYNC 1  /* Algorithm 1 (C-Syn): read L, atomic-min into L_u, L = L_u */

/* Driver: how sweeps are sequenced. */
#define CONTOUR_DRIVER_PERSISTENT 0 /* one launch; workgroups pull edge chunks from a task
                                       counter and open the next sweep on device */
#define CONTOUR_DRIVER_HOSTLOOP 1   /* one launch per sweep; the host reads the convergence
                                       word every few sweeps (this call blocks) */

typedef struct {
    int32_t order;       /* 0 = default (2); 1..CONTOUR_ORDER_MAX or CONTOUR_ORDER_FULL */
    int32_t schedule;    /* CONTOUR_SCHED_* */
    int32_t k1;          /* C-11mm: sweeps of order 1 before switching (0 = 2) */
    int32_t write_mode;  /* CONTOUR_WRITE_* */
    int32_t update;      /* CONTOUR_UPDATE_* (SYNC requires DRIVER_HOSTLOOP) */
    int32_t driver;      /* CONTOUR_DRIVER_* */
    int32_t max_sweeps;  /* 0 = no limit */
    int32_t warm_start;  /* 1: labels_inout holds a state with L[x] <= x and L[x] in x's
                            component (e.g. a partial result); 0: start from L[x] = x */
    int32_t block;       /* threads per workgroup, 0 = auto; 256, 512 or 1024 */
    int32_t edges_per_thread; /* 0 = auto; 1, 2, 4 or 8 */
    int32_t chunk_tiles; /* persistent driver: tiles (block * edges_per_thread edges)
                            per task, 0 = auto */
    int32_t grid;        /* workgroups, 0 = auto (all resident) */
    int32_t reorder;     /* CONTOUR_REORDER_*: group the edges by source-vertex block
                            before the sweeps (a radix partition on device) */
    int32_t window;      /* with reordering: labels staged in LDS per task, 0 = as many
                            as one workgroup's LDS holds; at least 1024 */
    int32_t dst_ranges;  /* CONTOUR_DST_RANGES_*: with reordering, also group the edges by
                            destination range and give each XCD its own ranges */
} contour_opts_t;

/* Edge reordering.  The sweeps may apply MM^h to the edges in any order
 * (Section III-B-1 leaves the order of the asynchronous updates free), so the
 * library may first copy the edge list into a workspace grouped by blocks of
 * source ids: the label gathers of neighbouring edges then share cache lines.
 * The input arrays are never modified; labels are identical either way. */
#define CONTOUR_REORDER_AUTO 0 /* on when the label array exceeds the caches of one XCD */
#define CONTOUR_REORDER_OFF 1
#define CONTOUR_REORDER_ON 2

/* Destination ranges (persistent driver, with reordering).  A second, stable
 * grouping pass orders the grouped edges by destination range (ranges of
 * 2^19 ids, 2 MiB of labels, at most 64 ranges), and the sweep's tasks are
 * dealt to the eight XCDs by segments of consecutive ranges, so the
 * destination-side label gathers of an XCD stay in its own L2 while the
 * source side keeps its LDS window.  Labels are identical either way. */
#define CONTOUR_DST_RANGES_AUTO 0 /* on when the label array exceeds one XCD's L2 and m >= 4 n */
#define CONTOUR_DST_RANGES_OFF 1
#define CONTOUR_DST_RANGES_ON 2   /* values 16..30 also mean on, with ranges of 2^value ids */

typedef struct {
    int32_t status;             /* contour_status_t of the data checks */
    int32_t sweeps_executed;    /* sweeps run, including the final one that changed nothing */
    int32_t sweeps_with_writes; /* sweeps in which some edge changed a label */
    int32_t reserved;
} contour_stats_t;

/* Fill *opts with the defaults (order 0, i.e. 2 for a solve and the tuned
 * order in a batched plan; fixed schedule, plain writes, asynchronous update,
 * persistent driver, no sweep limit, automatic geometry). */
void contour_default_opts(contour_opts_t* opts);

/* contour_cc: labels_out[v] = minimum vertex id of v's component.
 *   src, dst    device int32[m], ids in [0, n)
 *   m           edge count, >= 0 (0: labels are the identity)
 *   n           vertex count, >= 0 (0: nothing is done)
 *   labels_out  device int32[n], written
 * Defaults of contour_default_opts; data errors are not reported (use
 * contour_cc_ex for stats).  Returns CONTOUR_OK or a synchronous error. */
int contour_cc(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
               int32_t* labels_out, contour_stream_t stream);

/* contour_cc_ex: as contour_cc with options and statistics.
 *   labels_inout  device int32[n]; read first when opts->warm_start, then written
 *   opts          NULL for defaults
 *   stats         NULL, or a device (or host-pinned) contour_stats_t written by the
 *                 device when the solve ends
 * Returns CONTOUR_OK, CONTOUR_EINVAL, CONTOUR_ENOTSUP, CONTOUR_ENOMEM or CONTOUR_EHIP. */
int contour_cc_ex(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                  int32_t* labels_inout, const contour_opts_t* opts, contour_stats_t* stats,
                  contour_stream_t stream);

/* contour_cc_count_reads: an instrumented contour_cc_ex (persistent driver)
 * that also counts the label reads of the operator's chains, for measuring
 * the traffic of operators whose reads per edge are not fixed.  For every
 * edge and sweep run with an order above 3 or CONTOUR_ORDER_FULL, the reads
 * of the chains w, L[w], ... and v, L[v], ... up to level h or to the root
 * (Definition 3; the reads that decide z and the early convergence check) are
 * added to *reads (device uint64, not cleared first).  Sweeps of orders 1..3
 * read exactly 2h labels per edge and are not counted.  The extra work is one
 * addition per read and one atomic per workgroup; labels and stats are those
 * of contour_cc_ex.  Returns as contour_cc_ex; CONTOUR_EINVAL for a NULL reads,
 * CONTOUR_ENOTSUP with the host-loop driver. */
int contour_cc_count_reads(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                           int32_t* labels_inout, const contour_opts_t* opts, contour_stats_t* stats,
                           uint64_t* reads, contour_stream_t stream);

/* contour_reserve: allocate, up front, the workspace that contour_cc,
 * contour_cc_ex (persistent driver) and contour_group_edges need on `stream`
 * for graphs of up to m edges and n vertices under `opts` (NULL: defaults):
 * the stream's control block and scratch (the grouped copy of the edges and
 * the grouping's count tables: about 8.5 m bytes when the options group the
 * edges, 16.5 m with destination ranges).  It blocks (it may synchronise the stream and allocate); later calls
 * on the stream within these sizes enqueue only kernels and may be captured.
 * Reserving less than the stream already holds keeps what it holds.
 * contour_cc_add_edges and the host-loop driver keep their own behaviour.
 * Returns CONTOUR_OK, CONTOUR_EINVAL, CONTOUR_ENOTSUP, CONTOUR_ENOMEM or
 * CONTOUR_EHIP. */
int contour_reserve(int64_t m, int32_t n, const contour_opts_t* opts, contour_stream_t stream);

/* contour_cc_noalloc: contour_cc_ex for callers that cannot allocate device
 * memory -- code under hipGraph stream capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It calls no hipMalloc, hipFree or allocating library
 * routine: the solve's scratch (its control block and, when the edges are
 * grouped, the grouped copy and the grouping's count tables) is one fixed
 * device array of CONTOUR_NOALLOC_SCRATCH_BYTES per device, held by the library
 * until the process ends.
 *   arguments   as contour_cc_ex (same meaning, layout and ownership)
 *   limits      the persistent driver only (CONTOUR_DRIVER_HOSTLOOP gives
 *               CONTOUR_ENOTSUP, and so does CONTOUR_UPDATE_SYNC, as for
 *               contour_cc_ex).  Grouping the edges needs about 8.5 m bytes of
 *               the array (8 m for the grouped copy, m / 2 for the count
 *               tables), so up to about 3.9 million edges are grouped (the
 *               second pass by destination range needs another 8 m and is
 *               left out under CONTOUR_DST_RANGES_AUTO when it does not fit): with
 *               CONTOUR_REORDER_AUTO a graph whose grouped copy does not fit is
 *               solved without grouping (same labels, slower); with
 *               CONTOUR_REORDER_ON it is refused with CONTOUR_ETOOBIG and nothing
 *               is enqueued.
 *   races       every call on one device shares that device's array, and each
 *               call resets it when its work starts on the device: calls whose
 *               work can overlap on one device (different streams, or host
 *               threads without ordering) race and give wrong results; calls on
 *               one stream are ordered by the stream.
 * Returns as contour_cc_ex, or CONTOUR_ETOOBIG. */
#define CONTOUR_NOALLOC_SCRATCH_BYTES (32u << 20)
int contour_cc_noalloc(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                       int32_t* labels_inout, const contour_opts_t* opts, contour_stats_t* stats,
                       contour_stream_t stream);

/* contour_group_edges: the edge list grouped by source block, as a solve that
 * reorders prepares it before its first sweep (the asynchronous update of
 * Algorithm 1 may take the edges in any order, Section III-B-1).
 *   src, dst          device int32[m], the edges
 *   m                 edge count, 0 <= m < 2^31 - 1 (0: nothing is done)
 *   n                 vertex count, > 0
 *   src_out, dst_out  device int32[m], written; must not overlap src or dst
 * The output holds the same (src, dst) pairs, unchanged.  They are ordered by
 * block b = min(src >> s, K - 1), src read as unsigned, where s is the
 * smallest shift with (n - 1) >> s < 1024 and K = ((n - 1) >> s) + 1 (so an
 * id outside [0, n) lands in block K - 1).  Within a block they follow the
 * chunks of 8192 consecutive input edges in input order; within one
 * (block, chunk) run the order is unspecified.  A workspace of about m / 8
 * ints is kept per (device, stream) and reused.  Returns CONTOUR_OK,
 * CONTOUR_EINVAL (negative or too large m, n <= 0, a NULL array with m > 0),
 * CONTOUR_ENOMEM or CONTOUR_EHIP. */
int contour_group_edges(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                        int32_t* src_out, int32_t* dst_out, contour_stream_t stream);

/* contour_group_edges_ranges: the edge list as a solve with destination
 * ranges prepares it: grouped by source block as above, then stably by
 * destination range r = min(dst >> t, R - 1), dst read as unsigned, where t is
 * the smallest shift >= 19 with (n - 1) >> t < 64 and R = ((n - 1) >> t) + 1.
 * The output lists the edges by range, within a range by source block, and
 * within one (range, block) by the 8192-edge chunks of the input in input
 * order.  Arguments, limits and returns as contour_group_edges, with n > 2^19
 * (smaller n: CONTOUR_EINVAL, there would be one range); a workspace of about
 * 8.5 m bytes is kept per (device, stream). */
int contour_group_edges_ranges(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                               int32_t* src_out, int32_t* dst_out, contour_stream_t stream);

/* contour_cc_add_edges: labels after adding edges to a labelled graph.
 *   src, dst      device int32[m], the new edges (ids in [0, n))
 *   m             new edge count, >= 0, at most (2^31 - 4) / 3
 *   labels_inout  device int32[n]: on entry the exact labels of some graph G on
 *                 the same n vertices (as returned by contour_cc / contour_cc_ex,
 *                 each vertex labelled with its component's minimum id); on
 *                 return the labels of G plus the new edges
 *   opts          NULL for defaults; warm_start is implied
 *   stats         as for contour_cc_ex
 * Not in the paper; it uses the property that any state with L[x] <= x and
 * L[x] in x's component is a valid start (Algorithm 1 only ever lowers labels
 * within a component, Section II-A).  Only the new edges are swept, each with
 * two ties (w, L[w]) and (v, L[v]) to the old roots of its endpoints, from the
 * old labels; every label is then replaced by the root of its chain.  The old
 * edges are never read, so the cost is O(m) per sweep plus O(n) for the final
 * pass.  Labels on entry that break 0 <= L[x] <= x are refused as for a warm
 * start of contour_cc_ex (stats status CONTOUR_EINVAL, labels unchanged); labels
 * that satisfy it but are not the exact labels of a graph give labels of some
 * coarser state, not an error.  A workspace of 6 m ints is kept per (device,
 * stream) and reused.  Returns as contour_cc_ex. */
int contour_cc_add_edges(const int32_t* src, const int32_t* dst, int64_t m, int32_t n,
                         int32_t* labels_inout, const contour_opts_t* opts, contour_stats_t* stats,
                         contour_stream_t stream);

/* ------------------------------------------------------------ batches -- */
/* A CSR-of-graphs batch of G independent graphs.  Graph g owns local vertex
 * ids 0..n_g-1 with n_g = vertex_offsets[g+1] - vertex_offsets[g] (< 2^31),
 * and edges edge_offsets[g] .. edge_offsets[g+1] of src/dst, written in local
 * ids.  Its labels (local minimum ids) land at labels_out + vertex_offsets[g].
 * Each graph's labels are independent of the rest of the batch. */
typedef struct {
    int32_t num_graphs;
    const int64_t* h_edge_offsets;   /* host int64[G+1], read at plan creation */
    const int64_t* h_vertex_offsets; /* host int64[G+1], read at plan creation */
    const int32_t* src;              /* device int32[edge_offsets[G]] */
    const int32_t* dst;              /* device int32[edge_offsets[G]] */
    int32_t* labels_out;             /* device int32[vertex_offsets[G]] */
    contour_stats_t* stats_out;      /* device contour_stats_t[G], or NULL */
} contour_batch_t;

typedef struct contour_plan* contour_plan_t;

/* Per-class choices of a batched plan.  Graphs fall into three classes:
 *   class 0  n <= lds_max_vertices: one workgroup solves the graph with its
 *            label array in LDS
 *   class 1  otherwise, m <= wg_max_edges: one workgroup solves the graph with
 *            its labels in global memory, the lowest ids (as many as the LDS
 *            holds) kept in LDS for the whole solve
 *   class 2  the rest: several workgroups per graph, sequenced on device by
 *            per-graph task counters (as the persistent driver)
 * Zero fields mean "automatic".  The autotuner in the Python package measures
 * candidates per class and produces this structure. */
typedef struct {
    int32_t order;            /* 0: from opts (default 2); 1..CONTOUR_ORDER_MAX or CONTOUR_ORDER_FULL */
    int32_t block;            /* 0: auto; 256, 512 (and 1024 for classes 0 and 1) */
    int32_t edges_per_thread; /* 0: auto; 1, 2, 4 or 8 */
    int32_t reserved;         /* must be 0 */
} contour_class_tuning_t;

typedef struct {
    contour_class_tuning_t cls[3];
    int32_t lds_max_vertices; /* class 0 bound, 0 or too large: as many labels as the LDS of one
                                 workgroup holds (about 40,000 on the MI355X); class-0 graphs above
                                 16384 vertices run in a launch of their own, with the class-0 order
                                 and 1024-thread workgroups of 4 edges per thread */
    int32_t wg_max_edges;     /* class 1 bound, 0: auto (2^19) */
} contour_batch_tuning_t;

/* Build a reusable plan: sorts the graphs into size classes (labels in LDS,
 * one workgroup per graph with labels in global memory, several workgroups
 * per graph), picks the per-class order and geometry, and allocates the
 * plan's device tables.  Non-zero opts->order, opts->block and
 * opts->edges_per_thread override the tuned choice for every class where the
 * value is allowed (block 1024 for classes 0 and 1, 8 edges per thread for
 * class 2); zero fields take the tuning table's choice, else the defaults.
 * opts->chunk_tiles, grid, reorder, window and dst_ranges do not apply to
 * plans.  The pointers in *batch are captured; the arrays they point to
 * must stay valid for launches.  Returns CONTOUR_OK, CONTOUR_EINVAL,
 * CONTOUR_ENOMEM or CONTOUR_EHIP. */
int contour_batch_plan_create(const contour_batch_t* batch, const contour_opts_t* opts,
                              contour_plan_t* plan_out);

/* As contour_batch_plan_create with explicit per-class choices (NULL: automatic). */
int contour_batch_plan_create_tuned(const contour_batch_t* batch, const contour_opts_t* opts,
                                    const contour_batch_tuning_t* tuning, contour_plan_t* plan_out);

/* Number of graphs of the plan in each class (counts[3]); CONTOUR_OK or EINVAL. */
int contour_batch_plan_classes(contour_plan_t plan, int32_t* counts);

/* Enqueue one solve of every graph of the plan on `stream`.  Enqueues only
 * kernels (no allocation, no host synchronisation, no memset), so it can be
 * captured into a hipGraph and replayed.  Returns CONTOUR_OK or CONTOUR_EHIP. */
int contour_batch_plan_launch(contour_plan_t plan, contour_stream_t stream);

/* Release a plan and its device tables (waits for the device). */
int contour_batch_plan_destroy(contour_plan_t plan);

/* Create, launch and destroy a plan in one call (blocks until done). */
int contour_cc_batched(const contour_batch_t* batch, const contour_opts_t* opts,
                       contour_stream_t stream);

/* -------------------------------------------------------- sharding ---- */
/* contour_merge_min: labels_inout[i] = min(labels_inout[i], peer[i]) for
 * every i in [0, n).  The combine step of an edge split of one graph over
 * several devices (not in the paper): each device sweeps its share of the
 * edges against a full copy of the labels, and the copies are merged by an
 * elementwise minimum.  In the pointer-graph view of the labels (Section
 * II-A) every label names a vertex of the same component at or below its own
 * id; the minimum of two such states keeps that and never raises a label, so
 * rounds of local solves and merges reach the unique fixed point, and a round
 * in which no solve changed a label and no merge lowered one is the last.
 *   peer          device int32[n], read
 *   labels_inout  device int32[n], updated in place; may be peer itself, must
 *                 not otherwise overlap it
 *   lowered       NULL, or device int32: set to the number of labels the
 *                 merge lowered
 * Enqueued on `stream`.  Returns CONTOUR_OK, CONTOUR_EINVAL (n < 0, a NULL
 * array with n > 0) or CONTOUR_EHIP. */
int contour_merge_min(const int32_t* peer, int32_t* labels_inout, int32_t n, int32_t* lowered,
                      contour_stream_t stream);

/* ------------------------------------------------------- profiling ---- */
/* contour_gather_ceiling: a measurement kernel, the memory access pattern of
 * a sweep without its arithmetic, for comparing a sweep's time with what the
 * GPU can do with the same accesses.  It reads src[0..m) and dst[0..m) once
 * and, with mode 1, gathers labels[dst[e]] for every edge (mode 2: also
 * labels[src[e]]), ids outside [0, n) skipped; the edge list is cut into
 * eight segments dealt to the eight XCDs, as the sweep's XCD queues deal a
 * copy grouped by destination range.  Nothing is written but, practically
 * never, sink[0] (device int32).  Enqueued on `stream`; time it with events.
 * Returns CONTOUR_OK, CONTOUR_EINVAL or CONTOUR_EHIP. */
int contour_gather_ceiling(const int32_t* src, const int32_t* dst, int64_t m, const int32_t* labels, int32_t n,
                           int32_t mode, int32_t* sink, contour_stream_t stream);


/* Optional timing hook for benchmarks.  When set (non-NULL hipEvent_t
 * handles), contour_cc / contour_cc_ex record `begin` on the call's stream
 * just before the first sweep kernel and `end` just after the last, so the
 * pair brackets exactly the sweep kernels (label initialisation and the
 * statistics write excluded).  The setting is per calling thread; pass NULL
 * twice to clear it.  The events are owned by the caller. */
void contour_set_timing_events(void* begin, void* end);

/* ------------------------------------------------------------- misc ---- */
const char* contour_status_string(int status);
int contour_last_hip_error(void);
const char* contour_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CONTOUR_H */
