// Structures shared by the host runtime and the gfx950 kernels.
#pragma once
#include <stdint.h>

namespace rs {

// Device control block of a batch (zero-initialised once).  A one-wave reset kernel runs
// before every launch of the pipeline kernel on the same stream: it zeroes the claim
// counters and advances the epoch, so a launch can be replayed (HIP graph) as is.
enum Ctl : uint32_t {
    CTL_ERROR = 2,          // watchdog / protocol error flag (sticky until read)
    CTL_EPOCH = 3,          // launch epoch (look-back state tags)
    CTL_BAD = 4,            // some stream of the batch has malformed regions (its ST_ERROR word says which)
    CTL_NPART = 64,         // claim partitions (8 per XCD); a launch uses 64, or 1 (the kernel relies on this)
    CTL_PART = 64,          // claim counter of partition q at CTL_PART + q * CTL_PART_STRIDE
    CTL_PART_STRIDE = 32,   // one 128-byte line per counter
    CTL_WORDS = CTL_PART + CTL_NPART * CTL_PART_STRIDE
};

// Statistics slots per stream (u64 each).
enum Stat : uint32_t {
    ST_FIRINGS = 0,    // [3]
    ST_ITEMS = 3,      // [3]
    ST_FULL = 6,       // [3]
    ST_SIGNALS = 9,    // [3]
    ST_OUTPUTS = 12,
    ST_ERROR = 15,     // low word: nonzero when a claim found malformed regions
    ST_WORDS = 16
};

// One stream of a batched launch (device work table entry).
struct StreamDev {
    const void *elements;
    const uint32_t *offsets;       // CSR [P+1] or starts [P]
    const uint32_t *lengths;       // nullptr for CSR
    const uint32_t *pparam;        // per-parent context or nullptr
    uint32_t *agg_count;
    unsigned long long *agg_sum;
    uint32_t *agg_min;
    uint32_t *agg_max;
    uint32_t *agg_kcount;          // tree: the second sink's count and sum, or nullptr
    unsigned long long *agg_ksum;
    uint32_t *out_items;           // ordered output stream or nullptr
    unsigned long long *lookback;  // per-claim look-back words (emit_outputs) or nullptr
    unsigned long long *stats;     // ST_WORDS counters or nullptr
    uint32_t n_parents;
    uint32_t n_elements;
    uint32_t parents_per_claim;    // B
    uint32_t n_claims;
    uint32_t claim_begin;          // first global claim index of this stream
    uint32_t pad[3];
};

struct LaunchArgs {
    const StreamDev *streams;
    uint32_t *ctl;
    uint32_t n_streams;
    uint32_t total_claims;
    uint32_t param[4];
    uint32_t agg_fields;
    uint32_t collect_stats;
    uint32_t emit_outputs;
    uint32_t bmax;                 // most parents in any claim of the launch (sizes the per-claim LDS)
    uint32_t n_parts;              // claim partitions: CTL_NPART, or 1 when claims must start in order
    uint32_t lb_wait_us;           // longest wait of one look-back step on a predecessor claim (microseconds)
    uint32_t qdepth;               // queue depth: a power of two in [2w, 8w] (data slots of the first queue)
};

// The no-allocation entry point (run_noalloc) keeps its device state in one static array of
// the kernel file: the control block, a table of at most NOALLOC_MAX_STREAMS streams and their
// statistics.  The table reaches the device as a kernel argument (no host staging buffer).
constexpr uint32_t NOALLOC_MAX_STREAMS = 16;
constexpr uint32_t NOALLOC_CTL_OFF = 0;
constexpr uint32_t NOALLOC_TABLE_OFF = 8448;   // CTL_WORDS * 4, a multiple of 256
constexpr uint32_t NOALLOC_TABLE_STRIDE = 256;   // bytes reserved per table entry (sizeof(StreamDev) at most)
constexpr uint32_t NOALLOC_STATS_OFF = NOALLOC_TABLE_OFF + NOALLOC_MAX_STREAMS * NOALLOC_TABLE_STRIDE;
constexpr uint32_t NOALLOC_SCRATCH_BYTES = NOALLOC_STATS_OFF + NOALLOC_MAX_STREAMS * 16 * 8;
struct NoallocTable {
    StreamDev s[NOALLOC_MAX_STREAMS];
    uint32_t n;
};

// Kernel entry points (defined in rs_kernels.hip).
// Lanes per workgroup of the kernel for ensemble width w (w = lanes * items per lane).
uint32_t lanes_of(uint32_t ensemble_width);
// Most parents one claim may hold (the region table has 256 entries, the last is the end offset).
inline uint32_t claim_parents_max(uint32_t ensemble_width) { return ensemble_width ? 255u : 0u; }
bool kernel_supported(uint32_t kind, uint32_t strategy, uint32_t width);
// Enqueues the reset kernel, then the pipeline kernel, on stream.  Non-null ev_begin/ev_end
// (HIP events) are recorded directly before and after the pipeline kernel.
int launch_pipeline(uint32_t kind, uint32_t strategy, uint32_t width, const LaunchArgs &a,
                    uint32_t grid, void *stream, void *ev_begin = nullptr, void *ev_end = nullptr);
int blocks_per_cu(uint32_t kind, uint32_t strategy, uint32_t width, uint32_t qdepth, uint32_t bmax);
// Bytes of dynamic LDS: the data queues for queue depth qdepth, and the per-claim arrays (region
// table and aggregate slots) for claims of up to bmax parents.
uint32_t dyn_lds_bytes(uint32_t kind, uint32_t strategy, uint32_t width, uint32_t qdepth, uint32_t bmax);
int launch_probe_copy(const void *src, void *dst, unsigned long long bytes, uint32_t n_cu, void *stream);
// Device address of the no-allocation scratch array on the current device (looked up once per
// device with hipGetSymbolAddress; the array itself is file-scope in rs_kernels.hip).
int noalloc_scratch(void **out);
// Clears the control block and the statistics in the scratch array at base and writes the stream
// table there, on stream.
int launch_noalloc_init(void *base, const NoallocTable &tab, void *stream);


}  // namespace rs
