/*
 * regionstream — region-stateful irregular streaming on MI355X (gfx950).
 *
 * C ABI of the library.  The computation is the enumeration-and-aggregation
 * dataflow of Timcheck & Buhler, "Streaming Computations with Region-Based
 * State on SIMD Architectures":
 *
 *   - enumeration (§4): a stream of parents (composite objects) is opened into
 *     the stream of their elements; each parent's elements form a region, and
 *     the element is fetched by index under its parent's context (§4.1);
 *   - irregular stages (§2.1): every stage maps one input to 0..k outputs,
 *     k known a priori per stage, the actual count data dependent;
 *   - aggregation (§4): each region's surviving items are reduced under that
 *     region's context, one record per parent (begin()/end() bracket every
 *     parent, §4.1), and optionally the survivors are emitted as a stream
 *     stripped of their parent context;
 *   - boundary transport: region boundaries reach every stage at exact stream
 *     positions either as signals with the credit protocol of §3.1-§3.3 (no
 *     ensemble mixes two regions, §3.3) or as a region tag carried by every
 *     item (the tagging alternative compared in §5).
 *
 * All arithmetic is integer: u32 items, u64 sums (mod 2^64), u32 counts,
 * minima and maxima.  Results are exactly those of the serial definition and
 * do not depend on strategy, ensemble width, queue depth, grid or batching.
 *
 * Every function returns RS_OK (0) or a negative rs_status; on failure
 * rs_last_error() returns a thread-local message.  Functions are not
 * reentrant for one pipeline; separate pipelines are independent.
 */
#ifndef REGIONSTREAM_H
#define REGIONSTREAM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RS_ABI_VERSION 1u

enum rs_status {
    RS_OK = 0,
    RS_EINVAL = -1,     /* bad argument or malformed stream (offsets, sizes, alignment) */
    RS_ENOMEM = -2,     /* device or host allocation failed */
    RS_EDEVICE = -3,    /* HIP error, or the device watchdog stopped a run */
    RS_EBUDGET = -4,    /* the stream alone exceeds the pipeline's HBM budget */
    RS_ENOTREADY = -5,  /* non-blocking read of a stream that has not finished */
    RS_ESTATE = -6,     /* call not valid in the stream's or pipeline's current state */
    RS_ENOTFOUND = -7   /* unknown stream id */
};

/* Boundary transport.  RS_SIGNAL: end-of-region signals on a finite signal queue beside each
 * data queue, delivered precisely with credit (§3.1-§3.3), so no ensemble spans a boundary;
 * RS_TAG: a region tag on every item (§5); RS_AUTO: the autotuner chooses;
 * RS_SIGNAL_LANES: the lane-resolved signals the paper proposes as future work (§6): the same
 * signal queues, but an ensemble may span boundaries and every node computes each lane's
 * region from the pending signals' positions instead of storing it with the items.  Offered for
 * u32 kinds (not RS_TEXT_WORDS) at ensemble widths 64, 128 and 256.
 * RS_ENUM_TAG: a choice per stage, the second version of the paper's taxi application (§5): the
 * enumerating stage works one region at a time, as under signals, and tags every item it emits
 * with that region, so the later stages work as under tags, their ensembles spanning regions.
 * Offered for the kinds with a second stage (RS_HASH_EXPAND, RS_HASH_TREE, RS_TEXT_WORDS).  The autotuner
 * therefore chooses per stage among signals on both edges (RS_SIGNAL), enumeration then tags
 * (RS_ENUM_TAG) and tags on both (RS_TAG), besides lane-resolved signals. */
enum rs_strategy { RS_TAG = 0, RS_SIGNAL = 1, RS_AUTO = 2, RS_SIGNAL_LANES = 3, RS_ENUM_TAG = 4 };

/* Stage kinds (hand-written HIP stages; there is no user device code).
 *   RS_MODFILTER    u32 elements; keep x mod param[0] == param[1] (param[0] 0 means 4); k = 1.
 *   RS_HASH_EXPAND  u32 elements; keep x when bit 0 of H(x,0) is set, then emit
 *                   c = (H(x,0) >> 1) & 3 children H(x, j+1), j ascending (k = 1, then 3);
 *                   H(x,s) = fmix32(x ^ 0x9E3779B9*(s+1)), fmix32 = MurmurHash3's finalizer.
 *   RS_TEXT_WORDS   byte elements, one region per line (starts + lengths); keep the
 *                   line-relative positions that start a word (a non-space byte at the line
 *                   start or after ' '), then map each start to its word length (k = 1, 1).
 *   RS_GRAPH_THRESH u32 edge weights grouped by source vertex; keep w < parent_param[src]
 *                   (strict); k = 1.
 *   RS_HASH_TREE    the stages of RS_HASH_EXPAND in a tree topology (§2.1, Fig. 1b): the filter
 *                   has two children, the expansion (whose children reach the aggregating node
 *                   of count/sum/min/max) and a second aggregating node that takes the filter's
 *                   survivors themselves (RS_KEPT_COUNT, RS_KEPT_SUM).  Region boundaries reach
 *                   both children as the strategy carries them.
 * The item that reaches aggregation is x, the child value, the word length or w. */
enum rs_kind { RS_MODFILTER = 1, RS_HASH_EXPAND = 2, RS_TEXT_WORDS = 3, RS_GRAPH_THRESH = 4, RS_HASH_TREE = 5 };

/* Aggregate fields; identities for a region without survivors: 0, 0, 0xFFFFFFFF, 0.  The last two
 * are the second sink of RS_HASH_TREE: per region, how many elements pass the filter and their
 * sum (u64). */
enum rs_aggf { RS_COUNT = 1, RS_SUM = 2, RS_MIN = 4, RS_MAX = 8, RS_KEPT_COUNT = 16, RS_KEPT_SUM = 32 };

enum rs_mem { RS_MEM_HOST = 0, RS_MEM_DEVICE = 1 };

/* run() flags */
#define RS_RUN_SYNC      0u   /* return after the launch has finished */
#define RS_RUN_ASYNC     1u   /* return after enqueueing on the pipeline's HIP stream */
#define RS_RUN_PER_STREAM 2u  /* one launch per stream instead of one batched launch */

/* serve() flags (besides RS_RUN_PER_STREAM) */
#define RS_SERVE_DEVICE_OUT 8u /* out[i] holds device arrays that the kernel writes directly */

/* read_*() flags */
#define RS_READ_BLOCK    0u
#define RS_NONBLOCK      1u   /* RS_ENOTREADY instead of waiting */
#define RS_READ_DEVICE   2u   /* the destination pointers are device memory */
#define RS_READ_RELEASE  4u   /* free the stream's device state after this read */

/* rs_pipeline_desc.flags */
#define RS_COLLECT_STATS 1u   /* count firings, items, full ensembles and signals per node */
#define RS_NO_GRAPH      2u   /* do not capture/replay the launch as a HIP graph */
#define RS_TIME_KERNEL   4u   /* time the pipeline kernel of every run with HIP events (kernel_times);
                                 implies RS_NO_GRAPH */

typedef struct rs_pipeline rs_pipeline;   /* opaque, library-owned */

/*
 * Pipeline description.
 *   abi_version     must be RS_ABI_VERSION
 *   kind            rs_kind
 *   strategy        rs_strategy
 *   agg_fields      OR of rs_aggf: the fields the pipeline stores (others are not written)
 *   ensemble_width  0 = autotune, else 64, 128, 256, 512 or 1024: the SIMD width w, the largest
 *                   ensemble one firing of a node consumes (§2.2; one wave64 processes w/64
 *                   items per lane per firing)
 *   queue_depth     0 = tuned with strategy and width when either is left to the autotuner
 *                   (2w or 4w), else 2w; otherwise a power of two in [2w, 8w]: the slots of the
 *                   queue in front of the second stage; the queue in front of the aggregating
 *                   stage holds as many, and one ensemble more behind the expansion (whose k = 3
 *                   worst case must fit above a leftover).  A node fires only when its downstream
 *                   queue has room for what the firing may produce (§3.2 fireability), so the
 *                   depth decides when nodes fire, never what they compute.  Refused when the
 *                   queues do not fit a compute unit's LDS at the width.
 *   emit_outputs    1 = also produce the ordered surviving-item stream (read_outputs)
 *   flags           RS_COLLECT_STATS | RS_NO_GRAPH | RS_TIME_KERNEL
 *   hbm_budget_bytes  0 = unlimited; else streams are admitted to a run only while the device
 *                   footprint of admitted streams stays within the budget
 *   param           stage parameters (RS_MODFILTER: modulus, residue)
 */
typedef struct {
    uint32_t abi_version;
    uint32_t kind;
    uint32_t strategy;
    uint32_t agg_fields;
    uint32_t ensemble_width;
    uint32_t queue_depth;
    uint32_t emit_outputs;
    uint32_t flags;
    uint64_t hbm_budget_bytes;
    uint32_t param[4];
} rs_pipeline_desc;

/*
 * One input stream: a sequence of parents and their elements (§4).
 *   mem           rs_mem of every pointer below
 *   elem_bytes    4 (u32 elements) or 1 (bytes, RS_TEXT_WORDS)
 *   n_parents     P (< 2^32)
 *   n_elements    size of the element array (< 2^32)
 *   offsets       lengths == NULL: CSR offsets [P+1], region p = [offsets[p], offsets[p+1]),
 *                 non-decreasing, offsets[P] <= n_elements;
 *                 lengths != NULL: region starts [P], region p = [offsets[p], offsets[p]+lengths[p]),
 *                 starts non-decreasing and regions disjoint (the text form: line starts and lengths, §5)
 *   elements      element array, 16-byte aligned
 *   parent_param  per-parent context [P] (RS_GRAPH_THRESH: threshold), else NULL
 * With RS_MEM_HOST the library copies the arrays at stream_push (outside any timed run).
 * With RS_MEM_DEVICE the pointers are borrowed and must stay valid until the stream's
 * read_aggregates returns; the host then checks sizes and alignment only.
 */
typedef struct {
    uint32_t mem;
    uint32_t elem_bytes;
    uint64_t n_parents;
    uint64_t n_elements;
    const uint32_t *offsets;
    const uint32_t *lengths;
    const void *elements;
    const uint32_t *parent_param;
} rs_stream_desc;

/* Destination of read_aggregates: per-parent arrays [P]; a NULL pointer skips that field. */
typedef struct {
    uint32_t *count;
    uint64_t *sum;
    uint32_t *min;
    uint32_t *max;
    uint32_t *kept_count;   /* RS_HASH_TREE's second sink */
    uint64_t *kept_sum;
} rs_agg_view;

/* Device counters of one stream (RS_COLLECT_STATS).  Node 0 is the enumerated first stage,
 * node 1 the second stage (if any), node 2 the aggregating stage.  "full" counts firings whose
 * ensemble held w items, the statistic of §5 (full ensembles 91% vs 9% of the time). */
typedef struct {
    uint64_t firings[3];
    uint64_t items[3];
    uint64_t full[3];
    uint64_t signals[3];
    uint32_t ensemble_width;
    uint32_t queue_depth;
    uint32_t strategy;
    uint32_t n_workgroups;
    uint64_t n_outputs;
} rs_stats_t;

/* Validate the description and create a pipeline: the application of §2.1, nodes joined by
 * fixed-size data queues, whose first node enumerates each parent into its elements (§4) and
 * whose last aggregates each region (§4.1), every node firing ensembles of at most w items
 * (§2.2).  Creates the pipeline's HIP streams (default priority) on the current device; device
 * memory is taken at stream_push and run.  *out is library-owned until pipeline_destroy.
 * Errors: RS_EINVAL (bad description), RS_ENOMEM, RS_EDEVICE. */
int pipeline_create(const rs_pipeline_desc *d, rs_pipeline **out);

/* Make the pipeline enqueue its work on the given HIP stream (hipStream_t) instead of its own;
 * NULL restores the pipeline's own stream.  Host plumbing, no passage of the paper.
 * Errors: RS_EINVAL. */
int pipeline_set_stream(rs_pipeline *p, void *hip_stream);

/* Register one input stream: a sequence of parents, each with its element count or range (the
 * findCount of §4; the text application of §5 is given line start indices and lengths) and an
 * optional per-parent context (getParent, §4.1).  Validates it (host memory: offsets monotone
 * and in range, in O(P)), copies host arrays to the device, allocates the aggregate arrays and
 * returns an id.
 * Errors: RS_EINVAL (malformed stream, with a message), RS_EBUDGET (larger than the whole
 * budget), RS_ENOMEM, RS_EDEVICE. */
int stream_push(rs_pipeline *p, const rs_stream_desc *s, uint64_t *stream_id);

/* Process every pushed stream that has not run yet: admitted streams (by budget) go into one
 * persistent launch in which one-wave processors take parent batches from per-XCD
 * partitions of the launch's claims, by index or from a partition counter, and the kernel
 * returns only when every claim is consumed (§2.2); streams that do not fit wait for the next
 * run().  RS_RUN_SYNC waits for completion.
 * Errors: RS_EDEVICE (HIP error or watchdog), RS_ESTATE (nothing to run is not an error: RS_OK). */
int run(rs_pipeline *p, uint32_t flags);

/* Launch the most recent batch again, in place, on the same streams (their results are
 * recomputed bit for bit).  Used to time steady-state runs; the launch is captured into a
 * HIP graph on first use and replayed, unless RS_NO_GRAPH or RS_COLLECT_STATS is set.
 * Errors: RS_ESTATE (no batch has run), RS_EDEVICE. */
int run_again(rs_pipeline *p, uint32_t flags);

/* Copy one stream's per-parent aggregates, the record end() emits for each region (§4.1,
 * begin/run/end bracket every parent, empty ones included), into caller-owned arrays (host
 * memory, or device memory with RS_READ_DEVICE).  Waits for the stream's run unless RS_NONBLOCK.
 * Errors: RS_ENOTFOUND, RS_ESTATE (stream never ran), RS_ENOTREADY, RS_EDEVICE. */
int read_aggregates(rs_pipeline *p, uint64_t stream_id, rs_agg_view *out, uint32_t flags);

/* Copy the ordered output stream, the survivors stripped of their parent context (§4), in serial
 * order (parent, element index, child index), of a pipeline created with emit_outputs = 1.  *n_out receives the full length; at most cap items
 * are written.  Errors as read_aggregates, plus RS_EINVAL when emit_outputs was 0. */
int read_outputs(rs_pipeline *p, uint64_t stream_id, uint32_t *out, uint64_t cap,
                 uint64_t *n_out, uint32_t flags);

/* Device statistics of one stream (zeros unless RS_COLLECT_STATS): firings, items and full
 * ensembles per node, the occupancy measure of §5 (full ensembles 91% vs 9% of firings).
 * Errors as read_aggregates. */
int rs_stats(rs_pipeline *p, uint64_t stream_id, rs_stats_t *out);

/* Measurement aid (pipelines created with RS_TIME_KERNEL): the device time of the pipeline
 * kernel of every run and run_again since the previous call, in launch order, in
 * milliseconds.  Each launch records a pair of HIP events on its own stream, directly before
 * and after the pipeline kernel (the small reset kernel in front of it is outside the pair);
 * this call waits for them.  At most cap values go to ms (caller-owned host memory, may be NULL
 * when cap is 0); *n receives how many launches were timed, and all of them are consumed.
 * Errors: RS_EINVAL (NULL p or n, or the pipeline lacks RS_TIME_KERNEL), RS_EDEVICE. */
int kernel_times(rs_pipeline *p, float *ms, uint32_t cap, uint32_t *n);

/* Free a finished stream's device state; its id becomes unknown.  Host plumbing, no passage of
 * the paper.  Errors: RS_ENOTFOUND, RS_ESTATE (still running). */
int stream_release(rs_pipeline *p, uint64_t stream_id);

/* One request of the serving loop: its input stream and when it arrives, in seconds after
 * serve() starts. */
typedef struct {
    double arrival_s;
    rs_stream_desc stream;
} rs_request;

/* Host clock of one request, in seconds after serve() starts: arrival, push (input copied and
 * registered), launch (its batch enqueued) and completion (its aggregates read back). */
typedef struct {
    double arrival_s;
    double pushed_s;
    double launched_s;
    double completed_s;
    uint64_t batch;           /* launch batch the request ran in */
    int32_t status;           /* RS_OK or the error of this request */
    uint32_t pad;
} rs_request_timing;

/* Serve a sequence of requests in real time (continuous batching, beyond the paper, whose
 * kernel consumes one input stream per launch, §2.2).  The loop pushes every
 * request whose arrival time has passed, admits pushed requests into a new batch whenever
 * one of the pipeline's two launch lanes is free and the HBM budget allows (requests that
 * do not fit wait for earlier ones to finish and release their memory), reaps finished
 * batches without blocking, copies each request's aggregates into out[i] (host memory;
 * out may be NULL, or out[i] fields NULL) and releases it.  With RS_SERVE_DEVICE_OUT, out[i]
 * instead holds device arrays of n_parents entries for every field of agg_fields (none NULL;
 * owned by the caller, untouched by the library once serve returns); the kernel writes the
 * aggregates there in place, so a finished request costs no copy, and the pipeline must not
 * emit an output stream.  With RS_RUN_PER_STREAM every
 * request is launched alone, in arrival order, on one lane: the one-launch-per-stream
 * baseline.  Requests are sorted by arrival by the caller.  timing[i] receives the
 * request's clock.  Returns RS_OK when every request completed; a request that fails
 * records its error in timing[i].status and the loop goes on.
 * Errors: RS_EINVAL (NULL arguments, unsorted arrivals, a NULL device destination). */
int serve(rs_pipeline *p, const rs_request *reqs, uint64_t n, rs_agg_view *out, rs_request_timing *timing,
          uint32_t flags);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): run(), for n_streams (1..16) device-resident streams
 * in one persistent launch, with no allocation of any kind.  The library's device state for the
 * call (control block, stream table, statistics: about 12 KB) lives in one static array per device,
 * held until the process ends; the caller passes inputs and outputs.
 *   d          as for pipeline_create, with an explicit strategy (not RS_AUTO) and ensemble width
 *              and emit_outputs = 0 (queue_depth 0 means 2w)
 *   streams    n_streams stream descriptions, mem = RS_MEM_DEVICE (borrowed until the launch ends)
 *   out        n_streams destinations: device arrays [n_parents] of every field in agg_fields
 *   hip_stream HIP stream the launch is enqueued on (NULL: the default stream)
 *   flags      RS_RUN_SYNC: wait and report device errors (watchdog, malformed regions);
 *              RS_RUN_ASYNC: return after enqueueing, device errors are not reported
 * Calls on one device share its array: calls that overlap on a device (different host threads
 * or HIP streams without ordering) race and give wrong results.  Each call clears what must start
 * at zero.  Results are bit-identical to pipeline_create/stream_push/run/read_aggregates with the
 * same strategy and width.
 * Errors: RS_EINVAL (bad description, more than 16 streams, host memory, NULL destination,
 * malformed regions), RS_EDEVICE. */
int run_noalloc(const rs_pipeline_desc *d, const rs_stream_desc *streams, uint32_t n_streams,
                rs_agg_view *out, void *hip_stream, uint32_t flags);

/* Measurement aid: copy `bytes` (a multiple of 16) from src to dst, both 16-byte aligned device
 * memory, with a plain grid-stride copy kernel enqueued on hip_stream (NULL: the default stream).
 * It is the achievable-bandwidth reference beside the pipeline kernels and the known-size copy
 * that calibrates hardware traffic counters.  Errors: RS_EINVAL, RS_EDEVICE. */
int hbm_probe(const void *src, void *dst, uint64_t bytes, void *hip_stream);

/* Wait for outstanding work and free everything the pipeline owns.  Borrowed memory is
 * untouched.  Host plumbing, no passage of the paper. */
int pipeline_destroy(rs_pipeline *p);

/* Message of the last failure on this thread ("" if none; a thread-local buffer the library
 * owns, valid until the thread's next call). */
const char *rs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* REGIONSTREAM_H */
