// Host runtime behind the C ABI (include/regionstream.h).
//
// A pipeline owns two HIP streams of default priority (or borrows the caller's), and
// the device state of its streams.  run() gathers every pushed stream that fits the
// HBM budget into one batch: a device work table plus its own control block, and one
// launch of the persistent kernel in which workgroups compete for parent batches
// through a device atomic and return only when every claim is done (§2.2).  Batches
// launched back to back alternate between the two HIP streams, so a new batch starts
// on compute units that the previous one's last claims no longer use.
//
// When the description leaves the strategy or the ensemble width open, the first
// run() times every candidate on the first stream of the batch and keeps the fastest
// (§5: the right mechanism depends on elements per region against the SIMD width;
// §6 asks for that choice to be made from measurement).  Choices are cached on disk
// per kind and mean-region-length bucket.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <thread>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <memory>
#include <string>
#include <vector>

#include "../../include/regionstream.h"
#include "rs_internal.h"

#define RS_API extern "C" __attribute__((visibility("default")))

namespace {

// message of the last failure on this thread (a fixed buffer: recording an error allocates nothing)
thread_local char g_err[512];

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

void clear_error() { g_err[0] = '\0'; }

#define HIP_OR(expr, code)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(code, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

uint32_t k_max_of(uint32_t kind) { return kind == RS_HASH_EXPAND || kind == RS_HASH_TREE ? 3u : 1u; }
// aggregate fields a kind stores: the tree adds its second sink's
uint32_t fields_of(uint32_t kind) { return kind == RS_HASH_TREE ? 63u : 15u; }
uint32_t elem_bytes_of(uint32_t kind) { return kind == RS_TEXT_WORDS ? 1u : 4u; }

const uint32_t kWidths[] = {64, 128, 256, 512, 1024};

// Look-back words carry the batch's launch count modulo 2^24 - 1 as a tag.
constexpr uint64_t kEpochCycle = 0xFFFFFFull;

enum StreamState { S_PUSHED = 0, S_LAUNCHED = 1, S_DONE = 2 };

// Device blocks are recycled through a process-wide cache by size class instead of being given
// back with hipFree, which waits for the whole device: a serving loop that releases a finished
// stream would otherwise stall behind every launch still running.  Classes are 4 KiB, then four
// steps per power of two (at most 25% rounding).  The cache is emptied when the last pipeline is
// destroyed, and before an allocation that fails is retried.
class BlockCache {
  public:
    static size_t class_of(size_t n) {
        if (n <= 4096) return 4096;
        size_t top = 4096;
        while (top < n) top <<= 1;
        const size_t q = top >> 3;   // quarter steps between top/2 and top
        size_t c = top >> 1;
        while (c < n) c += q;
        return c;
    }
    int get(size_t n, void **out, size_t *cls, int *dev) {
        HIP_OR(hipGetDevice(dev), RS_EDEVICE);
        *cls = class_of(n);
        {
            std::lock_guard<std::mutex> g(mu_);
            auto it = free_.find({*dev, *cls});
            if (it != free_.end() && !it->second.empty()) {
                *out = it->second.back();
                it->second.pop_back();
                cached_ -= *cls;
                return RS_OK;
            }
        }
        hipError_t e = hipMalloc(out, *cls);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim();
            e = hipMalloc(out, *cls);
        }
        if (e != hipSuccess) {
            *out = nullptr;
            return fail(RS_ENOMEM, "hipMalloc(%zu): %s", *cls, hipGetErrorString(e));
        }
        return RS_OK;
    }
    void put(void *p, size_t cls, int dev) {
        std::lock_guard<std::mutex> g(mu_);
        free_[{dev, cls}].push_back(p);
        cached_ += cls;
    }
    // Returns every cached block with hipFree (callers know no kernel uses them).
    void trim() {
        std::map<std::pair<int, size_t>, std::vector<void *>> all;
        {
            std::lock_guard<std::mutex> g(mu_);
            all.swap(free_);
            cached_ = 0;
        }
        int cur = 0;
        (void)hipGetDevice(&cur);
        for (auto &kv : all) {
            (void)hipSetDevice(kv.first.first);
            for (void *p : kv.second) (void)hipFree(p);
        }
        (void)hipSetDevice(cur);
    }

  private:
    std::mutex mu_;
    std::map<std::pair<int, size_t>, std::vector<void *>> free_;
    size_t cached_ = 0;
};

BlockCache &block_cache() {
    static BlockCache *c = new BlockCache;   // outlives static destructors that might still free
    return *c;
}
int g_live_pipelines = 0;
std::mutex g_live_mu;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;   // bytes asked for
    size_t cls = 0;     // bytes held (the size class)
    int dev = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { reset(); }
    void reset() {
        if (p) block_cache().put(p, cls, dev);
        p = nullptr;
        bytes = cls = 0;
    }
    int alloc(size_t n) {
        reset();
        if (n == 0) n = 16;
        const int rc = block_cache().get(n, &p, &cls, &dev);
        if (rc) return rc;
        bytes = n;
        return RS_OK;
    }
};

struct Batch;

struct Stream {
    uint64_t id = 0;
    StreamState state = S_PUSHED;
    uint32_t n_parents = 0, n_elements = 0;
    double mean_len = 0;
    const void *elements = nullptr;
    const uint32_t *offsets = nullptr, *lengths = nullptr, *pparam = nullptr;
    DevBuf own_elements, own_offsets, own_lengths, own_pparam;
    DevBuf count, sum, min, max, kcount, ksum, stats;
    DevBuf out, lookback;          // ordered output stream and its per-claim look-back words
    uint64_t out_cap = 0;
    uint32_t B = 1, n_claims = 0;  // parents per claim and claims, planned at launch
    uint64_t footprint = 0;
    uint64_t batch = 0;            // batch this stream runs in
    hipEvent_t ready = nullptr;    // its host-to-device copies have landed (pushes that do not wait)
    rs_agg_view direct{};          // caller's device arrays the kernel writes directly (serve with RS_SERVE_DEVICE_OUT)
    bool has_direct = false;
    ~Stream() {
        if (ready) (void)hipEventDestroy(ready);
    }
};

struct Batch {
    std::vector<uint64_t> ids;
    std::vector<rs::StreamDev> host_table;   // source of the table's copy, kept until the batch is freed
    DevBuf table, ctl;
    uint32_t total_claims = 0;
    uint32_t grid = 0;
    uint32_t strategy = 0, width = 0, qdepth = 0;
    rs::LaunchArgs args{};
    hipStream_t lane = nullptr;
    uint64_t launches = 0;         // launches of this batch (its control block counts them too)
    uint64_t checked = ~0ull;      // launch count at which err_word and bad_word were read
    uint32_t err_word = 0, bad_word = 0;
    hipGraphExec_t graph = nullptr;
    hipEvent_t done = nullptr;
    ~Batch() {
        // the table and control block go back to the block cache after this body: the last
        // launch must have finished reading them
        if (done && launches) (void)hipEventSynchronize(done);
        if (graph) (void)hipGraphExecDestroy(graph);
        if (done) (void)hipEventDestroy(done);
    }
};

}  // namespace

struct rs_pipeline {
    rs_pipeline_desc d{};
    int device = 0;
    int n_cu = 0;
    hipStream_t own[2] = {nullptr, nullptr};
    hipStream_t copy = nullptr;    // host-to-device copies of pushed streams, apart from the launch lanes
    hipStream_t user_stream = nullptr;
    bool one_lane = false;         // every batch on the first lane (the per-stream baseline)
    uint32_t width = 0, strategy = 0, qdepth = 0;
    bool configured = false;
    uint64_t next_id = 1, next_batch = 1;
    uint64_t admitted_bytes = 0;
    std::map<uint64_t, std::unique_ptr<Stream>> streams;
    std::map<uint64_t, std::unique_ptr<Batch>> batches;
    uint64_t last_batch = 0;
    // RS_TIME_KERNEL: event pairs around launched pipeline kernels (oldest first), and spares
    std::deque<std::pair<hipEvent_t, hipEvent_t>> timed, spare_events;
};

namespace {

// ---------------------------------------------------------------- autotune cache

std::string cache_path() {
    if (const char *e = getenv("RS_AUTOTUNE_CACHE")) return e;
    const char *xdg = getenv("XDG_CACHE_HOME");
    const char *home = getenv("HOME");
    std::string dir = xdg ? std::string(xdg) : home ? std::string(home) + "/.cache" : std::string("/tmp");
    return dir + "/regionstream-autotune-gfx950-v2.txt";
}

int length_bucket(double mean_len) { return (int)std::lround(2.0 * std::log2(std::max(mean_len, 0.5))); }

bool depth_ok(uint32_t width, uint32_t q) { return q && !(q & (q - 1)) && q >= 2 * width && q <= 8 * width; }

// The last cached choice for (kind, emit, bucket) that agrees with what the pipeline fixed itself
// (want_*: a strategy, width or depth, or RS_AUTO / 0 for free), so that pipelines of different
// fixed strategies keep their own tuned choices side by side.
bool cache_lookup(uint32_t kind, uint32_t emit, int bucket, uint32_t want_s, uint32_t want_w, uint32_t want_q,
                  uint32_t *strategy, uint32_t *width, uint32_t *depth) {
    FILE *f = fopen(cache_path().c_str(), "r");
    if (!f) return false;
    unsigned k, e, s, w, q;
    int b;
    bool found = false;
    while (fscanf(f, "%u %u %d %u %u %u", &k, &e, &b, &s, &w, &q) == 6) {
        if (k == kind && e == emit && b == bucket && s != RS_AUTO && rs::kernel_supported(k, s, w) && depth_ok(w, q) &&
            (want_s == RS_AUTO || want_s == s) && (want_w == 0 || want_w == w) && (want_q == 0 || want_q == q)) {
            *strategy = s;
            *width = w;
            *depth = q;
            found = true;   // the last line for a key wins
        }
    }
    fclose(f);
    return found;
}

void cache_store(uint32_t kind, uint32_t emit, int bucket, uint32_t strategy, uint32_t width, uint32_t depth) {
    FILE *f = fopen(cache_path().c_str(), "a");
    if (!f) return;
    fprintf(f, "%u %u %d %u %u %u\n", kind, emit, bucket, strategy, width, depth);
    fclose(f);
}

// ---------------------------------------------------------------- validation

int check_stream(const rs_pipeline *p, const rs_stream_desc *s) {
    if (!s) return fail(RS_EINVAL, "stream description is NULL");
    if (s->mem != RS_MEM_HOST && s->mem != RS_MEM_DEVICE) return fail(RS_EINVAL, "mem must be RS_MEM_HOST or RS_MEM_DEVICE");
    const uint32_t eb = elem_bytes_of(p->d.kind);
    if (s->elem_bytes != eb) return fail(RS_EINVAL, "elem_bytes must be %u for this kind", eb);
    if (s->n_parents >= (1ull << 32)) return fail(RS_EINVAL, "n_parents must be < 2^32");
    if (s->n_elements * eb > 0xFFFFFF00ull)
        return fail(RS_EINVAL, "stream of %llu bytes exceeds the 4 GiB addressing limit",
                    (unsigned long long)(s->n_elements * eb));
    if (s->n_parents && !s->offsets) return fail(RS_EINVAL, "offsets is NULL");
    if (s->n_elements && !s->elements) return fail(RS_EINVAL, "elements is NULL");
    if (p->d.kind == RS_GRAPH_THRESH && s->n_parents && !s->parent_param)
        return fail(RS_EINVAL, "RS_GRAPH_THRESH needs parent_param (per-vertex thresholds)");
    if (s->mem == RS_MEM_DEVICE && ((uintptr_t)s->elements & 15u))
        return fail(RS_EINVAL, "device element array must be 16-byte aligned");
    const uint64_t P = s->n_parents;
    if (s->mem == RS_MEM_HOST && P) {
        if (!s->lengths) {
            for (uint64_t i = 0; i < P; ++i)
                if (s->offsets[i + 1] < s->offsets[i])
                    return fail(RS_EINVAL, "offsets decrease at parent %llu", (unsigned long long)i);
            if (s->offsets[P] > s->n_elements)
                return fail(RS_EINVAL, "offsets[%llu] = %u exceeds n_elements", (unsigned long long)P, s->offsets[P]);
        } else {
            uint64_t prev_end = 0;
            for (uint64_t i = 0; i < P; ++i) {
                const uint64_t st = s->offsets[i], en = st + s->lengths[i];
                if (st < prev_end)
                    return fail(RS_EINVAL, "region %llu starts before the previous one ends", (unsigned long long)i);
                if (en > s->n_elements) return fail(RS_EINVAL, "region %llu ends past n_elements", (unsigned long long)i);
                prev_end = en;
            }
        }
    }
    return RS_OK;
}

hipStream_t lane_of(rs_pipeline *p, uint64_t batch_id) {
    return p->user_stream ? p->user_stream : p->own[p->one_lane ? 0 : (batch_id & 1)];
}

// ---------------------------------------------------------------- batches

// Claim size: about 16 ensembles of elements per claim, at most claim_parents_max(w)
// parents, at least one parent.  Over u32 elements a claim takes about 32 ensembles when the
// stream still makes enough such claims: at least 8192 (two for each of the about 4096 waves a
// launch keeps resident) for aggregation, where each claim's fixed cost (its region table, its
// records, its first copy) then falls on twice the elements, provided the claim keeps to 32
// parents (more parents mean larger per-claim LDS arrays and fewer resident waves); at least
// 2048 (8 per compute unit) for an ordered output stream, whose claims start in index order and
// each wait on its predecessor's output offset, so that fewer, larger claims shorten that chain.
// Text lines, whose lengths vary widely, and smaller streams keep 16.
void claim_plan(uint32_t kind, bool ordered_out, uint32_t width, uint32_t n_parents, double mean_len, uint32_t *B,
                uint32_t *n_claims) {
    const double bmax = rs::claim_parents_max(width);
    const double min_claims = ordered_out ? 2048.0 : 8192.0;
    const bool big = kind != RS_TEXT_WORDS && mean_len > 0 && (ordered_out || 32.0 * width / mean_len <= 32.0) &&
                     (double)n_parents * mean_len >= min_claims * 32.0 * width;
    double b = mean_len > 0 ? (big ? 32.0 : 16.0) * width / mean_len : bmax;
    // text lines hold few second-stage items (word starts) for their bytes: a claim takes at least
    // 8 lines while that leaves 2048 claims, so that the second stage's ensembles can fill up
    // across lines where the strategy lets them (tags)
    if (kind == RS_TEXT_WORDS) b = std::max(b, std::min(8.0, n_parents / 2048.0));
    *B = (uint32_t)std::max(1.0, std::min(bmax, b));
    *n_claims = (uint32_t)(((uint64_t)n_parents + *B - 1) / *B);
}

void plan_claims(Stream *s, uint32_t kind, bool ordered_out, uint32_t width, uint32_t n_parents) {
    claim_plan(kind, ordered_out, width, n_parents, s->mean_len, &s->B, &s->n_claims);
}

// Longest wait of one look-back step on a predecessor claim before the claim gives up and the
// launch reports a device error: 2 s, far beyond any healthy wait (a predecessor publishes its
// count within microseconds of starting).  RS_LOOKBACK_WAIT_US overrides it, so that tests can
// drive the give-up path.
uint32_t lookback_wait_us() {
    if (const char *e = getenv("RS_LOOKBACK_WAIT_US")) {
        char *end = nullptr;
        const unsigned long v = strtoul(e, &end, 10);
        if (end != e && v <= 0xFFFFFFFFul) return (uint32_t)v;
    }
    return 2000000u;
}

int make_batch(rs_pipeline *p, const std::vector<Stream *> &sel, uint64_t batch_id, bool probe,
               std::unique_ptr<Batch> &out) {
    std::unique_ptr<Batch> b(new Batch);
    b->strategy = p->strategy;
    b->width = p->width;
    b->qdepth = p->qdepth;
    b->lane = lane_of(p, batch_id);
    std::vector<rs::StreamDev> &h = b->host_table;
    h.resize(sel.size());
    uint64_t claims = 0;
    uint32_t bmax = 1;
    for (size_t i = 0; i < sel.size(); ++i) {
        Stream *s = sel[i];
        uint32_t P = s->n_parents;
        // probe on a prefix of about 2^25 elements, so the timing ranks configurations as the
        // full stream would.  A lone stream's prefix also holds claims for two per wave at 32
        // waves per compute unit under the widest candidate's claim plan (so every candidate
        // times the same prefix): with fewer the probe leaves compute units idle and hides what
        // larger queues and ensembles cost in resident waves (long regions, e.g. long text lines,
        // give few claims per 2^25 elements)
        if (probe && s->n_elements > (1u << 25) && P > 1) {
            const uint32_t P0 = P;
            P = (uint32_t)std::max<uint64_t>(1, (uint64_t)((double)P * (double)(1u << 25) / s->n_elements));
            if (sel.size() == 1) {
                uint32_t B = 1, nc = 0;
                claim_plan(p->d.kind, false, kWidths[sizeof kWidths / sizeof kWidths[0] - 1], P, s->mean_len, &B, &nc);
                const uint64_t want = 64ull * (uint64_t)std::max(1, p->n_cu);
                if (nc < want) P = (uint32_t)std::min<uint64_t>(P0, (uint64_t)P * want / std::max<uint32_t>(1, nc) + 1);
            }
        }
        plan_claims(s, p->d.kind, p->d.emit_outputs && !probe, p->width, P);
        rs::StreamDev &e = h[i];
        std::memset(&e, 0, sizeof e);
        e.elements = s->elements;
        e.offsets = s->offsets;
        e.lengths = s->lengths;
        e.pparam = s->pparam;
        if (s->has_direct) {
            e.agg_count = s->direct.count;
            e.agg_sum = (unsigned long long *)s->direct.sum;
            e.agg_min = s->direct.min;
            e.agg_max = s->direct.max;
            e.agg_kcount = s->direct.kept_count;
            e.agg_ksum = (unsigned long long *)s->direct.kept_sum;
        } else {
            e.agg_count = (uint32_t *)s->count.p;
            e.agg_sum = (unsigned long long *)s->sum.p;
            e.agg_min = (uint32_t *)s->min.p;
            e.agg_max = (uint32_t *)s->max.p;
            e.agg_kcount = (uint32_t *)s->kcount.p;
            e.agg_ksum = (unsigned long long *)s->ksum.p;
        }
        e.stats = (unsigned long long *)s->stats.p;   // the error word is always written
        if (p->d.emit_outputs && !probe) {
            const size_t lb_bytes = 8ull * s->n_claims + 8;
            if (s->lookback.bytes < lb_bytes) {
                int rc = s->lookback.alloc(lb_bytes);
                if (rc) return rc;
            }
            HIP_OR(hipMemsetAsync(s->lookback.p, 0, s->lookback.bytes, b->lane), RS_EDEVICE);
            e.out_items = (uint32_t *)s->out.p;
            e.lookback = (unsigned long long *)s->lookback.p;
        }
        e.n_parents = P;
        e.n_elements = s->n_elements;
        e.parents_per_claim = s->B;
        bmax = std::max(bmax, std::min(s->B, P));
        e.n_claims = s->n_claims;
        e.claim_begin = (uint32_t)claims;
        claims += s->n_claims;
        b->ids.push_back(s->id);
    }
    if (claims >= (1ull << 32) - (1ull << 20)) return fail(RS_EINVAL, "too many claims in one batch");
    int rc = b->table.alloc(sizeof(rs::StreamDev) * std::max<size_t>(1, h.size()));
    if (rc) return rc;
    if ((rc = b->ctl.alloc(rs::CTL_WORDS * sizeof(uint32_t)))) return rc;
    HIP_OR(hipMemsetAsync(b->ctl.p, 0, rs::CTL_WORDS * sizeof(uint32_t), b->lane), RS_EDEVICE);
    HIP_OR(hipMemcpyAsync(b->table.p, h.data(), sizeof(rs::StreamDev) * h.size(), hipMemcpyHostToDevice, b->lane),
           RS_EDEVICE);
    // the launch waits on the device, not the host, for streams whose copies are still landing
    for (Stream *s : sel)
        if (s->ready) HIP_OR(hipStreamWaitEvent(b->lane, s->ready, 0), RS_EDEVICE);
    HIP_OR(hipEventCreateWithFlags(&b->done, hipEventDisableTiming), RS_EDEVICE);
    b->total_claims = (uint32_t)claims;
    const int per_cu = rs::blocks_per_cu(p->d.kind, p->strategy, p->width, p->qdepth, bmax);
    if (per_cu <= 0) return fail(RS_EDEVICE, "kernel does not fit on a compute unit");
    // every workgroup holds two claims at a time (the next one's region table is prefetched)
    b->grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((claims + 1) / 2, (uint64_t)per_cu * p->n_cu));
    rs::LaunchArgs &a = b->args;
    a.streams = (const rs::StreamDev *)b->table.p;
    a.ctl = (uint32_t *)b->ctl.p;
    a.n_streams = (uint32_t)sel.size();
    a.total_claims = b->total_claims;
    std::memcpy(a.param, p->d.param, sizeof a.param);
    a.agg_fields = p->d.agg_fields;
    a.collect_stats = (!probe && (p->d.flags & RS_COLLECT_STATS)) ? 1u : 0u;
    a.emit_outputs = (!probe && p->d.emit_outputs) ? 1u : 0u;
    a.bmax = bmax;
    // the ordered output stream's look-back needs claims taken in index order, from one counter
    a.n_parts = a.emit_outputs ? 1u : rs::CTL_NPART;
    a.lb_wait_us = lookback_wait_us();
    a.qdepth = p->qdepth;
    out = std::move(b);
    return RS_OK;
}

// Clear look-back words whose tags could repeat on this launch.
int prepare_lookback(rs_pipeline *p, Batch &b) {
    if (!b.args.emit_outputs || b.launches == 0 || b.launches % kEpochCycle != 0) return RS_OK;
    for (uint64_t id : b.ids) {
        auto it = p->streams.find(id);
        if (it != p->streams.end() && it->second->lookback.p)
            HIP_OR(hipMemsetAsync(it->second->lookback.p, 0, it->second->lookback.bytes, b.lane), RS_EDEVICE);
    }
    return RS_OK;
}

// A pair of timing events, reused once kernel_times has read it.
int timing_events(rs_pipeline *p, std::pair<hipEvent_t, hipEvent_t> *ev) {
    if (!p->spare_events.empty()) {
        *ev = p->spare_events.front();
        p->spare_events.pop_front();
        return RS_OK;
    }
    HIP_OR(hipEventCreate(&ev->first), RS_EDEVICE);
    if (hipEventCreate(&ev->second) != hipSuccess) {
        (void)hipEventDestroy(ev->first);
        return fail(RS_EDEVICE, "hipEventCreate failed");
    }
    return RS_OK;
}

// timed: a run of the caller's (not an autotune probe) on a pipeline with RS_TIME_KERNEL
int launch_batch(rs_pipeline *p, Batch &b, bool graph, bool timed = false) {
    if (!b.total_claims) {
        HIP_OR(hipEventRecord(b.done, b.lane), RS_EDEVICE);
        return RS_OK;
    }
    int rc = prepare_lookback(p, b);
    if (rc) return rc;
    timed = timed && (p->d.flags & RS_TIME_KERNEL);
    if (timed) {
        std::pair<hipEvent_t, hipEvent_t> ev;
        if ((rc = timing_events(p, &ev))) return rc;
        rc = rs::launch_pipeline(p->d.kind, b.strategy, b.width, b.args, b.grid, b.lane, ev.first, ev.second);
        if (rc) {
            p->spare_events.push_back(ev);
            return fail(RS_EDEVICE, "kernel launch failed: %s", hipGetErrorString((hipError_t)rc));
        }
        p->timed.push_back(ev);
    } else if (graph) {
        if (!b.graph) {
            hipGraph_t g = nullptr;
            HIP_OR(hipStreamBeginCapture(b.lane, hipStreamCaptureModeThreadLocal), RS_EDEVICE);
            const int lrc = rs::launch_pipeline(p->d.kind, b.strategy, b.width, b.args, b.grid, b.lane);
            hipError_t e = hipStreamEndCapture(b.lane, &g);
            if (lrc || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(RS_EDEVICE, "graph capture failed");
            }
            e = hipGraphInstantiate(&b.graph, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail(RS_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
        }
        HIP_OR(hipGraphLaunch(b.graph, b.lane), RS_EDEVICE);
    } else {
        rc = rs::launch_pipeline(p->d.kind, b.strategy, b.width, b.args, b.grid, b.lane);
        if (rc) return fail(RS_EDEVICE, "kernel launch failed: %s", hipGetErrorString((hipError_t)rc));
    }
    ++b.launches;
    HIP_OR(hipEventRecord(b.done, b.lane), RS_EDEVICE);
    return RS_OK;
}

// Reads the control block's error and malformed-region words once per finished launch (the
// caller has waited for it); a batch's streams are then checked without a copy each.
int batch_error(Batch &b) {
    if (b.checked != b.launches) {
        uint32_t w[3] = {0, 0, 0};
        static_assert(rs::CTL_BAD == rs::CTL_ERROR + 2, "control words read together");
        HIP_OR(hipMemcpy(w, (uint32_t *)b.ctl.p + rs::CTL_ERROR, sizeof w, hipMemcpyDeviceToHost), RS_EDEVICE);
        b.err_word = w[0];
        b.bad_word = w[2];
        b.checked = b.launches;
    }
    if (b.err_word) return fail(RS_EDEVICE, "the device scheduler stopped a claim (watchdog or internal check)");
    return RS_OK;
}

// Time every candidate configuration on a probe batch that stands for the selection and keep the
// fastest (a runner-up within 5% is timed again beside it, and the second timing decides).  One launch runs one configuration for all of its streams, so the probe is the
// selection itself, or, above about 2^25 elements, every k-th stream of it in push order (each
// stream probed on a prefix of about 2^25 elements, a lone stream's prefix lengthened until it
// fills the grid with claims): a mix of short- and long-region streams
// is tuned as a mix.  The cache key is the probe's mean region length, kept apart for mixes.
int autotune(rs_pipeline *p, const std::vector<Stream *> &sel) {
    constexpr uint64_t kProbeElems = 1ull << 25;
    uint64_t total = 0;
    for (Stream *s : sel) total += s->n_elements;
    std::vector<Stream *> probe;
    const size_t step = total > kProbeElems ? (size_t)std::min<uint64_t>(sel.size(), total / kProbeElems + 1) : 1;
    for (size_t i = 0; i < sel.size(); i += step) probe.push_back(sel[i]);
    double covered = 0, parents = 0;
    for (Stream *s : probe) {
        covered += s->mean_len * s->n_parents;
        parents += s->n_parents;
    }
    const int bucket = length_bucket(parents > 0 ? covered / parents : 0.0) + (sel.size() > 1 ? 1000 : 0);
    const uint32_t want_s = p->d.strategy, want_w = p->d.ensemble_width, want_q = p->d.queue_depth;
    uint32_t cs = 0, cw = 0, cq = 0;
    if (cache_lookup(p->d.kind, p->d.emit_outputs, bucket, want_s, want_w, want_q, &cs, &cw, &cq)) {
        p->strategy = cs;
        p->width = cw;
        p->qdepth = cq;
        return RS_OK;
    }
    struct Cand {
        uint32_t s, w, q;
        float ms;
    };
    Cand c1{want_s == RS_AUTO ? (uint32_t)RS_TAG : want_s, want_w ? want_w : 256u, 0u, 1e30f};
    c1.q = want_q ? want_q : 2 * c1.w;
    Cand c2 = c1;   // the fastest and the runner-up
    hipEvent_t e0, e1;
    HIP_OR(hipEventCreate(&e0), RS_EDEVICE);
    HIP_OR(hipEventCreate(&e1), RS_EDEVICE);
    // one configuration on the probe: a warm-up, then the fastest of reps timed launches (one slow
    // launch, from another process or a clock change, does not decide the pick)
    auto time_cfg = [&](uint32_t strat, uint32_t w, uint32_t q, int reps, float *out) -> int {
        p->strategy = strat;
        p->width = w;
        p->qdepth = q;
        std::unique_ptr<Batch> b;
        int r = make_batch(p, probe, 0, true, b);
        if (r) return r;
        if ((r = launch_batch(p, *b, false))) return r;
        float ms = 1e30f;
        for (int i = 0; i < reps; ++i) {
            if (hipEventRecord(e0, b->lane) != hipSuccess) return fail(RS_EDEVICE, "event record");
            if ((r = launch_batch(p, *b, false))) return r;
            if (hipEventRecord(e1, b->lane) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
                return fail(RS_EDEVICE, "event synchronize");
            float one = 0;
            (void)hipEventElapsedTime(&one, e0, e1);
            ms = std::min(ms, one);
        }
        if ((r = batch_error(*b))) return r;
        *out = ms;
        return RS_OK;
    };
    int rc = RS_OK;
    for (uint32_t strat : {(uint32_t)RS_TAG, (uint32_t)RS_SIGNAL, (uint32_t)RS_SIGNAL_LANES, (uint32_t)RS_ENUM_TAG}) {
        if (rc != RS_OK) break;
        if (want_s != RS_AUTO && strat != want_s) continue;
        for (uint32_t wq = 0; wq < 2 * (sizeof kWidths / sizeof kWidths[0]) && rc == RS_OK; ++wq) {
            // every width at queue depths 2w and 4w (or at the depth asked for)
            const uint32_t w = kWidths[wq / 2];
            if (want_w && w != want_w) continue;
            if (!rs::kernel_supported(p->d.kind, strat, w)) continue;
            if (want_q && (wq % 2 || !depth_ok(w, want_q))) continue;
            const uint32_t q = want_q ? want_q : (wq % 2 ? 4 * w : 2 * w);
            // the queues and a full claim's arrays must fit a compute unit's LDS
            if (rs::blocks_per_cu(p->d.kind, strat, w, q, rs::claim_parents_max(w)) <= 0) continue;
            float ms = 1e30f;
            if ((rc = time_cfg(strat, w, q, 3, &ms))) break;
            if (ms < c1.ms) {
                c2 = c1;
                c1 = Cand{strat, w, q, ms};
            } else if (ms < c2.ms) {
                c2 = Cand{strat, w, q, ms};
            }
        }
    }
    // a close call (runner-up within 5%) is timed again, six launches each, and decided on that
    if (rc == RS_OK && c1.ms < 1e30f && c2.ms < 1.05f * c1.ms) {
        float m1 = 1e30f, m2 = 1e30f;
        if ((rc = time_cfg(c1.s, c1.w, c1.q, 6, &m1)) == RS_OK && (rc = time_cfg(c2.s, c2.w, c2.q, 6, &m2)) == RS_OK &&
            m2 < m1)
            c1 = c2;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    const uint32_t best_s = c1.s, best_w = c1.w, best_q = c1.q;
    p->strategy = best_s;
    p->width = best_w;
    p->qdepth = best_q;
    cache_store(p->d.kind, p->d.emit_outputs, bucket, best_s, best_w, best_q);
    return RS_OK;
}

int find_done(rs_pipeline *p, uint64_t id, uint32_t flags, Stream **out) {
    auto it = p->streams.find(id);
    if (it == p->streams.end()) return fail(RS_ENOTFOUND, "unknown stream id %llu", (unsigned long long)id);
    Stream *s = it->second.get();
    if (s->state == S_PUSHED) return fail(RS_ESTATE, "stream %llu has not been run", (unsigned long long)id);
    auto bi = p->batches.find(s->batch);
    if (bi == p->batches.end()) return fail(RS_ESTATE, "stream %llu has no batch", (unsigned long long)id);
    Batch &b = *bi->second;
    if (flags & RS_NONBLOCK) {
        hipError_t e = hipEventQuery(b.done);
        if (e == hipErrorNotReady) return fail(RS_ENOTREADY, "stream %llu is still running", (unsigned long long)id);
        if (e != hipSuccess) return fail(RS_EDEVICE, "hipEventQuery: %s", hipGetErrorString(e));
    } else {
        HIP_OR(hipEventSynchronize(b.done), RS_EDEVICE);
    }
    int rc = batch_error(b);
    if (rc) return rc;
    uint32_t bad = 0;
    if (b.bad_word)
        HIP_OR(hipMemcpy(&bad, (unsigned long long *)s->stats.p + rs::ST_ERROR, 4, hipMemcpyDeviceToHost), RS_EDEVICE);
    if (bad) return fail(RS_EINVAL, "stream %llu has malformed regions (out of order or past n_elements)",
                         (unsigned long long)id);
    s->state = S_DONE;
    *out = s;
    return RS_OK;
}

void release(rs_pipeline *p, Stream *s) {
    p->admitted_bytes -= std::min(p->admitted_bytes, s->footprint);
    const uint64_t bid = s->batch;
    p->streams.erase(s->id);
    // a batch whose streams are all gone is freed too
    auto bi = p->batches.find(bid);
    if (bi != p->batches.end()) {
        bool any = false;
        for (uint64_t id : bi->second->ids) any |= p->streams.count(id) > 0;
        if (!any && bid != p->last_batch) p->batches.erase(bi);
    }
}

}  // namespace

// ------------------------------------------------------------------------------ ABI

RS_API const char *rs_last_error(void) { return g_err; }

RS_API int pipeline_create(const rs_pipeline_desc *d, rs_pipeline **out) {
    clear_error();
    if (!d || !out) return fail(RS_EINVAL, "NULL argument");
    *out = nullptr;
    if (d->abi_version != RS_ABI_VERSION)
        return fail(RS_EINVAL, "abi_version %u, library is %u", d->abi_version, RS_ABI_VERSION);
    if (d->kind < RS_MODFILTER || d->kind > RS_HASH_TREE) return fail(RS_EINVAL, "unknown kind %u", d->kind);
    if (d->strategy > RS_ENUM_TAG) return fail(RS_EINVAL, "unknown strategy %u", d->strategy);
    if (d->strategy == RS_ENUM_TAG && !rs::kernel_supported(d->kind, RS_ENUM_TAG, d->ensemble_width ? d->ensemble_width : 64))
        return fail(RS_EINVAL, "enumeration with tags downstream is offered for kinds with a second stage");
    if (d->strategy == RS_SIGNAL_LANES && !rs::kernel_supported(d->kind, RS_SIGNAL_LANES, d->ensemble_width ? d->ensemble_width : 64))
        return fail(RS_EINVAL, "lane-resolved signals are offered for u32 kinds only");
    if (d->agg_fields == 0 || (d->agg_fields & ~fields_of(d->kind)))
        return fail(RS_EINVAL, "agg_fields must be a non-empty OR of RS_COUNT|RS_SUM|RS_MIN|RS_MAX "
                               "(and RS_KEPT_COUNT|RS_KEPT_SUM for RS_HASH_TREE)");
    const uint32_t w = d->ensemble_width;
    if (w && !rs::kernel_supported(d->kind, RS_TAG, w))
        return fail(RS_EINVAL, "ensemble_width %u not supported (64, 128, 256, 512 or 1024)", w);
    if (w && d->strategy == RS_SIGNAL_LANES && !rs::kernel_supported(d->kind, RS_SIGNAL_LANES, w))
        return fail(RS_EINVAL, "lane-resolved signals take ensemble_width 64, 128 or 256");
    if (d->queue_depth) {
        const uint32_t q = d->queue_depth;
        if (q & (q - 1)) return fail(RS_EINVAL, "queue_depth must be a power of two");
        if (w && !depth_ok(w, q))
            return fail(RS_EINVAL, "queue_depth %u must lie in [2w, 8w] = [%u, %u]", q, 2 * w, 8 * w);
        if (!w && (q < 128 || q > 8192))
            return fail(RS_EINVAL, "queue_depth %u fits no ensemble width (2w <= depth <= 8w)", q);
        if (w && d->strategy != RS_AUTO &&
            rs::blocks_per_cu(d->kind, d->strategy, w, q, rs::claim_parents_max(w)) <= 0)
            return fail(RS_EINVAL, "queue_depth %u: the queues do not fit a compute unit's LDS at this width", q);
    }
    if (d->emit_outputs > 1) return fail(RS_EINVAL, "emit_outputs must be 0 or 1");
    if (d->flags & ~7u) return fail(RS_EINVAL, "unknown pipeline flags");
    if (d->kind == RS_MODFILTER && d->param[0] != 0 && d->param[1] >= d->param[0])
        return fail(RS_EINVAL, "residue must be smaller than the modulus");

    std::unique_ptr<rs_pipeline> p(new rs_pipeline);
    p->d = *d;
    HIP_OR(hipGetDevice(&p->device), RS_EDEVICE);
    hipDeviceProp_t prop;
    HIP_OR(hipGetDeviceProperties(&prop, p->device), RS_EDEVICE);
    p->n_cu = prop.multiProcessorCount;
    for (auto &h : p->own) HIP_OR(hipStreamCreateWithFlags(&h, hipStreamNonBlocking), RS_EDEVICE);
    HIP_OR(hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking), RS_EDEVICE);
    {
        std::lock_guard<std::mutex> g(g_live_mu);
        ++g_live_pipelines;
    }
    p->width = d->ensemble_width;
    p->strategy = d->strategy == RS_AUTO ? RS_TAG : d->strategy;
    // queue_depth 0: twice the width when strategy and width are given, else tuned with them
    p->qdepth = d->queue_depth ? d->queue_depth : 2 * d->ensemble_width;
    p->configured = d->ensemble_width != 0 && d->strategy != RS_AUTO;
    *out = p.release();
    return RS_OK;
}

RS_API int pipeline_set_stream(rs_pipeline *p, void *hip_stream) {
    if (!p) return fail(RS_EINVAL, "NULL pipeline");
    p->user_stream = (hipStream_t)hip_stream;
    return RS_OK;
}

namespace {
int push_stream(rs_pipeline *p, const rs_stream_desc *s, uint64_t *stream_id, bool wait,
                const rs_agg_view *direct = nullptr);
}

RS_API int stream_push(rs_pipeline *p, const rs_stream_desc *s, uint64_t *stream_id) {
    return push_stream(p, s, stream_id, true);
}

namespace {
// wait: return after the copies have landed, so the caller may reuse its host arrays; else the
// stream's launch waits for them on the device (serve(), whose requests outlive the loop).
// direct: device arrays of the caller that receive the aggregates in place of the stream's own.
int push_stream(rs_pipeline *p, const rs_stream_desc *s, uint64_t *stream_id, bool wait,
                const rs_agg_view *direct) {
    clear_error();
    if (!p || !stream_id) return fail(RS_EINVAL, "NULL argument");
    int rc = check_stream(p, s);
    if (rc) return rc;
    std::unique_ptr<Stream> st(new Stream);
    st->n_parents = (uint32_t)s->n_parents;
    st->n_elements = (uint32_t)s->n_elements;
    const bool text = p->d.kind == RS_TEXT_WORDS;
    const uint32_t eb = elem_bytes_of(p->d.kind);
    const uint64_t P = s->n_parents;

    // region form expected by the kernels: CSR for u32 kinds, starts + lengths for text
    std::vector<uint32_t> conv_a, conv_b;
    const uint32_t *offs = s->offsets, *lens = s->lengths;
    if (s->mem == RS_MEM_HOST && P) {
        if (text && !lens) {
            conv_a.assign(offs, offs + P);
            conv_b.resize(P);
            for (uint64_t i = 0; i < P; ++i) conv_b[i] = offs[i + 1] - offs[i];
            offs = conv_a.data();
            lens = conv_b.data();
        } else if (!text && lens) {
            conv_a.resize(P + 1);
            for (uint64_t i = 0; i < P; ++i) {
                if (i && offs[i] != offs[i - 1] + lens[i - 1])
                    return fail(RS_EINVAL, "u32 kinds need contiguous regions (region %llu)", (unsigned long long)i);
                conv_a[i] = offs[i];
            }
            conv_a[P] = offs[P - 1] + lens[P - 1];
            offs = conv_a.data();
            lens = nullptr;
        }
    } else if (P && (text != (lens != nullptr))) {
        return fail(RS_EINVAL, text ? "device text streams need starts + lengths" : "device u32 streams need CSR offsets");
    }

    // mean region length sizes claims and keys the autotuner
    double covered = (double)s->n_elements;
    if (s->mem == RS_MEM_HOST && P) {
        covered = 0;
        if (lens) {
            for (uint64_t i = 0; i < P; ++i) covered += lens[i];
        } else {
            covered = (double)offs[P] - (double)offs[0];
        }
    }
    st->mean_len = P ? covered / (double)P : 0.0;

    // device footprint (look-back words at one per parent at most)
    const uint64_t agg_bytes = direct ? 0 : P * ((p->d.agg_fields & RS_COUNT ? 4 : 0) + (p->d.agg_fields & RS_SUM ? 8 : 0) +
                                    (p->d.agg_fields & RS_MIN ? 4 : 0) + (p->d.agg_fields & RS_MAX ? 4 : 0) +
                                    (p->d.agg_fields & RS_KEPT_COUNT ? 4 : 0) + (p->d.agg_fields & RS_KEPT_SUM ? 8 : 0));
    uint64_t in_bytes = 0;
    if (s->mem == RS_MEM_HOST)
        in_bytes = s->n_elements * eb + (lens ? 8 * P : 4 * (P + 1)) + (s->parent_param ? 4 * P : 0);
    st->out_cap = p->d.emit_outputs ? (uint64_t)k_max_of(p->d.kind) * s->n_elements : 0;
    const uint64_t est_claims = P ? std::max<uint64_t>(1, (uint64_t)(covered / (16.0 * 64))) + P / 64 + 1 : 0;
    st->footprint = in_bytes + agg_bytes + 8 * rs::ST_WORDS + 4 * st->out_cap +
                    (p->d.emit_outputs ? 8ull * std::min<uint64_t>(est_claims, P + 1) : 0);
    if (p->d.hbm_budget_bytes && st->footprint > p->d.hbm_budget_bytes)
        return fail(RS_EBUDGET, "stream needs %llu bytes, budget is %llu", (unsigned long long)st->footprint,
                    (unsigned long long)p->d.hbm_budget_bytes);

    // copies go on the pipeline's copy stream: a push does not wait for running launches
    hipStream_t hs = p->copy;
    if (s->mem == RS_MEM_HOST) {
        if ((rc = st->own_elements.alloc(s->n_elements * eb + 16))) return rc;
        if (s->n_elements)
            HIP_OR(hipMemcpyAsync(st->own_elements.p, s->elements, s->n_elements * eb, hipMemcpyHostToDevice, hs),
                   RS_EDEVICE);
        st->elements = st->own_elements.p;
        if (P) {
            const size_t ob = lens ? 4 * P : 4 * (P + 1);
            if ((rc = st->own_offsets.alloc(ob))) return rc;
            HIP_OR(hipMemcpyAsync(st->own_offsets.p, offs, ob, hipMemcpyHostToDevice, hs), RS_EDEVICE);
            st->offsets = (const uint32_t *)st->own_offsets.p;
            if (lens) {
                if ((rc = st->own_lengths.alloc(4 * P))) return rc;
                HIP_OR(hipMemcpyAsync(st->own_lengths.p, lens, 4 * P, hipMemcpyHostToDevice, hs), RS_EDEVICE);
                st->lengths = (const uint32_t *)st->own_lengths.p;
            }
            if (s->parent_param) {
                if ((rc = st->own_pparam.alloc(4 * P))) return rc;
                HIP_OR(hipMemcpyAsync(st->own_pparam.p, s->parent_param, 4 * P, hipMemcpyHostToDevice, hs), RS_EDEVICE);
                st->pparam = (const uint32_t *)st->own_pparam.p;
            }
        }
    } else {
        st->elements = s->elements;
        st->offsets = s->offsets;
        st->lengths = s->lengths;
        st->pparam = s->parent_param;
        // borrowed regions are checked by the kernel, claim by claim, before any element is read
    }
    if (direct) {
        st->direct = *direct;
        st->has_direct = true;
    } else {
        if (p->d.agg_fields & RS_COUNT && (rc = st->count.alloc(4 * P))) return rc;
        if (p->d.agg_fields & RS_SUM && (rc = st->sum.alloc(8 * P))) return rc;
        if (p->d.agg_fields & RS_MIN && (rc = st->min.alloc(4 * P))) return rc;
        if (p->d.agg_fields & RS_MAX && (rc = st->max.alloc(4 * P))) return rc;
        if (p->d.agg_fields & RS_KEPT_COUNT && (rc = st->kcount.alloc(4 * P))) return rc;
        if (p->d.agg_fields & RS_KEPT_SUM && (rc = st->ksum.alloc(8 * P))) return rc;
    }
    if ((rc = st->stats.alloc(8 * rs::ST_WORDS))) return rc;
    HIP_OR(hipMemsetAsync(st->stats.p, 0, 8 * rs::ST_WORDS, hs), RS_EDEVICE);
    if (wait) {
        // the copies and the clear have landed before any launch reads them, and the caller may
        // reuse its host arrays as soon as this returns
        HIP_OR(hipStreamSynchronize(hs), RS_EDEVICE);
    } else {
        HIP_OR(hipEventCreateWithFlags(&st->ready, hipEventDisableTiming), RS_EDEVICE);
        HIP_OR(hipEventRecord(st->ready, hs), RS_EDEVICE);
    }
    if (p->d.emit_outputs && (rc = st->out.alloc(4 * st->out_cap + 16))) return rc;

    st->id = p->next_id++;
    *stream_id = st->id;
    p->streams[st->id] = std::move(st);
    return RS_OK;
}
}  // namespace

namespace {

// Launch the given pushed streams: one batch, or one batch per stream.
int launch_streams(rs_pipeline *p, const std::vector<Stream *> &sel, bool per_stream, bool sync) {
    if (sel.empty()) return RS_OK;
    int rc;
    if (!p->configured) {
        if ((rc = autotune(p, sel))) return rc;
        p->configured = true;
    }
    std::vector<std::vector<Stream *>> groups;
    if (per_stream) {
        for (Stream *s : sel) groups.push_back({s});
    } else {
        groups.push_back(sel);
    }
    std::vector<Batch *> launched;
    for (auto &grp : groups) {
        const uint64_t bid = p->next_batch++;
        std::unique_ptr<Batch> b;
        if ((rc = make_batch(p, grp, bid, false, b))) return rc;
        if ((rc = launch_batch(p, *b, false, true))) return rc;
        for (Stream *s : grp) {
            s->state = S_LAUNCHED;
            s->batch = bid;
            p->admitted_bytes += s->footprint;
        }
        launched.push_back(b.get());
        p->batches[bid] = std::move(b);
        p->last_batch = bid;
    }
    if (sync) {
        for (Batch *b : launched) {
            HIP_OR(hipEventSynchronize(b->done), RS_EDEVICE);
            if ((rc = batch_error(*b))) return rc;
        }
    }
    return RS_OK;
}

// Pushed streams, in push order, that fit the HBM budget next to what is admitted.
std::vector<Stream *> admissible(rs_pipeline *p, const std::vector<Stream *> &cands, size_t limit) {
    std::vector<Stream *> sel;
    uint64_t used = p->admitted_bytes;
    for (Stream *s : cands) {
        if (sel.size() >= limit) break;
        if (s->state != S_PUSHED) continue;
        if (p->d.hbm_budget_bytes && used + s->footprint > p->d.hbm_budget_bytes) continue;
        used += s->footprint;
        sel.push_back(s);
    }
    return sel;
}

}  // namespace

RS_API int run(rs_pipeline *p, uint32_t flags) {
    clear_error();
    if (!p) return fail(RS_EINVAL, "NULL pipeline");
    if (flags & ~3u) return fail(RS_EINVAL, "unknown run flags");
    std::vector<Stream *> cands;
    for (auto &kv : p->streams) cands.push_back(kv.second.get());
    return launch_streams(p, admissible(p, cands, (size_t)-1), flags & RS_RUN_PER_STREAM, !(flags & RS_RUN_ASYNC));
}

RS_API int run_again(rs_pipeline *p, uint32_t flags) {
    clear_error();
    if (!p) return fail(RS_EINVAL, "NULL pipeline");
    if (flags & ~1u) return fail(RS_EINVAL, "unknown run flags");
    auto it = p->batches.find(p->last_batch);
    if (it == p->batches.end()) return fail(RS_ESTATE, "no batch has run on this pipeline");
    Batch &b = *it->second;
    if (p->user_stream) b.lane = p->user_stream;
    const bool graph = !(p->d.flags & (RS_NO_GRAPH | RS_COLLECT_STATS | RS_TIME_KERNEL));
    int rc = launch_batch(p, b, graph, true);
    if (rc) return rc;
    for (uint64_t id : b.ids) {
        auto si = p->streams.find(id);
        if (si != p->streams.end()) si->second->state = S_LAUNCHED;
    }
    if (!(flags & RS_RUN_ASYNC)) {
        HIP_OR(hipEventSynchronize(b.done), RS_EDEVICE);
        return batch_error(b);
    }
    return RS_OK;
}

RS_API int read_aggregates(rs_pipeline *p, uint64_t stream_id, rs_agg_view *out, uint32_t flags) {
    clear_error();
    if (!p || !out) return fail(RS_EINVAL, "NULL argument");
    if (flags & ~7u) return fail(RS_EINVAL, "unknown read flags");
    Stream *s = nullptr;
    int rc = find_done(p, stream_id, flags, &s);
    if (rc) return rc;
    const hipMemcpyKind k = (flags & RS_READ_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t P = s->n_parents;
    struct F {
        void *dst;
        DevBuf *src;
        size_t bytes;
        uint32_t bit;
        const char *name;
    };
    F fields[6] = {{out->count, &s->count, 4 * P, RS_COUNT, "count"},
                   {out->sum, &s->sum, 8 * P, RS_SUM, "sum"},
                   {out->min, &s->min, 4 * P, RS_MIN, "min"},
                   {out->max, &s->max, 4 * P, RS_MAX, "max"},
                   {out->kept_count, &s->kcount, 4 * P, RS_KEPT_COUNT, "kept_count"},
                   {out->kept_sum, &s->ksum, 8 * P, RS_KEPT_SUM, "kept_sum"}};
    for (auto &f : fields) {
        if (!f.dst) continue;
        if (!(p->d.agg_fields & f.bit)) return fail(RS_EINVAL, "field %s is not stored by this pipeline", f.name);
        if (P) HIP_OR(hipMemcpy(f.dst, f.src->p, f.bytes, k), RS_EDEVICE);
    }
    if (flags & RS_READ_RELEASE) release(p, s);
    return RS_OK;
}

RS_API int read_outputs(rs_pipeline *p, uint64_t stream_id, uint32_t *out, uint64_t cap, uint64_t *n_out,
                        uint32_t flags) {
    clear_error();
    if (!p || !n_out) return fail(RS_EINVAL, "NULL argument");
    if (!p->d.emit_outputs) return fail(RS_EINVAL, "pipeline was created without emit_outputs");
    Stream *s = nullptr;
    int rc = find_done(p, stream_id, flags, &s);
    if (rc) return rc;
    uint64_t n = 0;
    if (s->n_claims) {
        uint64_t w = 0;
        HIP_OR(hipMemcpy(&w, (uint64_t *)s->lookback.p + (s->n_claims - 1), 8, hipMemcpyDeviceToHost), RS_EDEVICE);
        if (((w >> 38) & 3u) != 2u)
            return fail(RS_EDEVICE, "output stream of stream %llu is incomplete", (unsigned long long)stream_id);
        n = w & ((1ull << 38) - 1ull);
    }
    *n_out = n;
    const uint64_t m = std::min<uint64_t>(n, cap);
    if (m) {
        if (!out) return fail(RS_EINVAL, "out is NULL");
        const hipMemcpyKind k = (flags & RS_READ_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
        HIP_OR(hipMemcpy(out, s->out.p, 4 * m, k), RS_EDEVICE);
    }
    if (flags & RS_READ_RELEASE) release(p, s);
    return RS_OK;
}

RS_API int rs_stats(rs_pipeline *p, uint64_t stream_id, rs_stats_t *out) {
    clear_error();
    if (!p || !out) return fail(RS_EINVAL, "NULL argument");
    Stream *s = nullptr;
    int rc = find_done(p, stream_id, 0, &s);
    if (rc) return rc;
    unsigned long long st[rs::ST_WORDS];
    HIP_OR(hipMemcpy(st, s->stats.p, sizeof st, hipMemcpyDeviceToHost), RS_EDEVICE);
    std::memset(out, 0, sizeof *out);
    for (int k = 0; k < 3; ++k) {
        out->firings[k] = st[rs::ST_FIRINGS + k];
        out->items[k] = st[rs::ST_ITEMS + k];
        out->full[k] = st[rs::ST_FULL + k];
        out->signals[k] = st[rs::ST_SIGNALS + k];
    }
    auto bi = p->batches.find(s->batch);
    if (bi != p->batches.end()) {
        out->ensemble_width = bi->second->width;
        out->queue_depth = bi->second->qdepth;
        out->strategy = bi->second->strategy;
        out->n_workgroups = bi->second->grid;
    }
    if (p->d.emit_outputs && s->n_claims && s->lookback.p) {
        uint64_t w = 0;
        HIP_OR(hipMemcpy(&w, (uint64_t *)s->lookback.p + (s->n_claims - 1), 8, hipMemcpyDeviceToHost), RS_EDEVICE);
        out->n_outputs = w & ((1ull << 38) - 1ull);
    }
    return RS_OK;
}

RS_API int stream_release(rs_pipeline *p, uint64_t stream_id) {
    clear_error();
    if (!p) return fail(RS_EINVAL, "NULL pipeline");
    auto it = p->streams.find(stream_id);
    if (it == p->streams.end()) return fail(RS_ENOTFOUND, "unknown stream id %llu", (unsigned long long)stream_id);
    Stream *s = it->second.get();
    if (s->state == S_LAUNCHED) {
        auto bi = p->batches.find(s->batch);
        if (bi != p->batches.end() && hipEventQuery(bi->second->done) == hipErrorNotReady)
            return fail(RS_ESTATE, "stream is still running");
        s->state = S_DONE;
    }
    release(p, s);
    return RS_OK;
}

RS_API int serve(rs_pipeline *p, const rs_request *reqs, uint64_t n, rs_agg_view *out, rs_request_timing *timing,
                 uint32_t flags) {
    clear_error();
    if (!p || (n && (!reqs || !timing))) return fail(RS_EINVAL, "NULL argument");
    if (flags & ~(RS_RUN_PER_STREAM | RS_SERVE_DEVICE_OUT)) return fail(RS_EINVAL, "unknown serve flags");
    const bool dev_out = flags & RS_SERVE_DEVICE_OUT;
    if (dev_out) {
        if (n && !out) return fail(RS_EINVAL, "RS_SERVE_DEVICE_OUT needs out");
        if (p->d.emit_outputs) return fail(RS_EINVAL, "RS_SERVE_DEVICE_OUT: the pipeline emits an output stream");
        for (uint64_t i = 0; i < n; ++i) {
            const rs_agg_view &o = out[i];
            const uint32_t f = p->d.agg_fields;
            if (reqs[i].stream.n_parents &&
                (((f & RS_COUNT) && !o.count) || ((f & RS_SUM) && !o.sum) || ((f & RS_MIN) && !o.min) ||
                 ((f & RS_MAX) && !o.max) || ((f & RS_KEPT_COUNT) && !o.kept_count) ||
                 ((f & RS_KEPT_SUM) && !o.kept_sum)))
                return fail(RS_EINVAL, "request %llu: a destination of a stored field is NULL", (unsigned long long)i);
        }
    }
    for (uint64_t i = 1; i < n; ++i)
        if (reqs[i].arrival_s < reqs[i - 1].arrival_s) return fail(RS_EINVAL, "requests must be sorted by arrival");
    const bool per_stream = flags & RS_RUN_PER_STREAM;
    struct LaneGuard {
        rs_pipeline *p;
        bool saved;
        ~LaneGuard() { p->one_lane = saved; }
    } lane_guard{p, p->one_lane};
    p->one_lane = per_stream;
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    auto now = [&]() { return std::chrono::duration<double>(clk::now() - t0).count(); };

    for (uint64_t i = 0; i < n; ++i) {
        std::memset(&timing[i], 0, sizeof timing[i]);
        timing[i].arrival_s = reqs[i].arrival_s;
    }
    std::vector<uint64_t> sid(n, 0);
    std::deque<uint64_t> waiting;                 // pushed, not yet launched (request indices)
    std::vector<uint64_t> inflight;               // launched, not yet completed
    uint64_t next = 0, done = 0;
    int last_rc = RS_OK;

    auto fail_req = [&](uint64_t i, int rc) {
        timing[i].status = rc;
        timing[i].completed_s = now();
        ++done;
        last_rc = rc;
    };
    while (done < n) {
        bool progressed = false;
        // 1. arrivals: push requests whose time has come, a few per pass so that launches and
        //    completions are not held up behind a long run of copies
        for (int pushed = 0; pushed < 4 && next < n && reqs[next].arrival_s <= now(); ++pushed) {
            uint64_t id = 0;
            // the launch waits for the copy on the device
            const int rc = push_stream(p, &reqs[next].stream, &id, false, dev_out ? &out[next] : nullptr);
            if (rc) {
                fail_req(next, rc);
            } else {
                sid[next] = id;
                timing[next].pushed_s = now();
                waiting.push_back(next);
            }
            ++next;
            progressed = true;
        }
        // 2. admission and launch: a new batch whenever a lane is free
        std::map<uint64_t, int> batches_inflight;
        for (uint64_t i : inflight) batches_inflight[timing[i].batch] = 1;
        // batched: a new batch whenever one of the two lanes is free; per stream: every
        // request is launched as soon as it is pushed and the lane runs them in order
        const size_t lanes = per_stream ? (size_t)-1 : 2;
        if (!waiting.empty() && batches_inflight.size() < lanes) {
            std::vector<Stream *> cands;
            for (uint64_t i : waiting) cands.push_back(p->streams.at(sid[i]).get());
            // per-stream baseline: one request per launch, in arrival order
            const std::vector<Stream *> sel = admissible(p, cands, per_stream ? 1 : (size_t)-1);
            const uint64_t before = p->next_batch;
            const int rc = launch_streams(p, sel, per_stream, false);
            if (rc) {
                while (!waiting.empty()) {
                    const uint64_t i = waiting.front();
                    waiting.pop_front();
                    (void)stream_release(p, sid[i]);
                    fail_req(i, rc);
                }
            } else if (p->next_batch != before) {
                std::deque<uint64_t> still;
                for (uint64_t i : waiting) {
                    Stream *s = p->streams.at(sid[i]).get();
                    if (s->state == S_LAUNCHED) {
                        timing[i].launched_s = now();
                        timing[i].batch = s->batch;
                        inflight.push_back(i);
                    } else {
                        still.push_back(i);   // over budget: waits for memory to free up
                    }
                }
                waiting.swap(still);
                progressed = true;
            }
        }
        // 3. completions: reap finished batches without blocking
        for (size_t k = 0; k < inflight.size();) {
            const uint64_t i = inflight[k];
            rs_agg_view dummy{};
            // device outputs are already in place: only the completion and the checks remain
            rs_agg_view *v = (out && !dev_out) ? &out[i] : &dummy;
            const int rc = read_aggregates(p, sid[i], v, RS_NONBLOCK | RS_READ_RELEASE);
            if (rc == RS_ENOTREADY) {
                ++k;
                continue;
            }
            if (rc) {
                (void)stream_release(p, sid[i]);
                fail_req(i, rc);
            } else {
                timing[i].completed_s = now();
                ++done;
            }
            inflight[k] = inflight.back();
            inflight.pop_back();
            progressed = true;
        }
        if (!progressed) {
            // nothing to do right now: wait for the next arrival or completion
            const double wait = next < n ? reqs[next].arrival_s - now() : 0.0;
            if (inflight.empty() && wait > 200e-6)
                std::this_thread::sleep_for(std::chrono::duration<double>(wait - 100e-6));
            else
                std::this_thread::sleep_for(std::chrono::microseconds(5));
        }
    }
    return last_rc == RS_OK ? RS_OK : fail(last_rc, "some requests failed (see timing[].status)");
}

RS_API int run_noalloc(const rs_pipeline_desc *d, const rs_stream_desc *streams, uint32_t n_streams,
                       rs_agg_view *out, void *hip_stream, uint32_t flags) {
    clear_error();
    // ---- everything is checked before the device is touched
    if (!d || !streams || !out) return fail(RS_EINVAL, "NULL argument");
    if (flags & ~RS_RUN_ASYNC) return fail(RS_EINVAL, "unknown run flags");
    if (n_streams == 0 || n_streams > rs::NOALLOC_MAX_STREAMS)
        return fail(RS_EINVAL, "run_noalloc takes 1 to %u streams per call (got %u)", rs::NOALLOC_MAX_STREAMS, n_streams);
    if (d->abi_version != RS_ABI_VERSION) return fail(RS_EINVAL, "abi_version %u, library is %u", d->abi_version, RS_ABI_VERSION);
    if (d->kind < RS_MODFILTER || d->kind > RS_HASH_TREE) return fail(RS_EINVAL, "unknown kind %u", d->kind);
    if (d->strategy == RS_AUTO || !rs::kernel_supported(d->kind, d->strategy, d->ensemble_width))
        return fail(RS_EINVAL, "run_noalloc needs an explicit strategy and ensemble width the kernels offer "
                               "(autotuning allocates)");
    if (d->agg_fields == 0 || (d->agg_fields & ~fields_of(d->kind)))
        return fail(RS_EINVAL, "agg_fields must be a non-empty OR of RS_COUNT|RS_SUM|RS_MIN|RS_MAX "
                               "(and RS_KEPT_COUNT|RS_KEPT_SUM for RS_HASH_TREE)");
    if (d->emit_outputs) return fail(RS_EINVAL, "run_noalloc does not produce the ordered output stream");
    const uint32_t qdepth = d->queue_depth ? d->queue_depth : 2 * d->ensemble_width;
    if (!depth_ok(d->ensemble_width, qdepth))
        return fail(RS_EINVAL, "queue_depth %u must be a power of two in [2w, 8w]", qdepth);
    if (d->kind == RS_MODFILTER && d->param[0] != 0 && d->param[1] >= d->param[0])
        return fail(RS_EINVAL, "residue must be smaller than the modulus");
    const bool text = d->kind == RS_TEXT_WORDS;
    const uint32_t eb = elem_bytes_of(d->kind);
    rs::NoallocTable tab;
    std::memset(&tab, 0, sizeof tab);
    static_assert(sizeof(rs::StreamDev) <= rs::NOALLOC_TABLE_STRIDE, "stream table entry");
    tab.n = n_streams;
    uint64_t claims = 0;
    uint32_t bmax = 1;
    for (uint32_t i = 0; i < n_streams; ++i) {
        const rs_stream_desc &s = streams[i];
        if (s.mem != RS_MEM_DEVICE) return fail(RS_EINVAL, "stream %u: run_noalloc takes device memory only", i);
        if (s.elem_bytes != eb) return fail(RS_EINVAL, "stream %u: elem_bytes must be %u for this kind", i, eb);
        if (s.n_parents >= (1ull << 32)) return fail(RS_EINVAL, "stream %u: n_parents must be < 2^32", i);
        if (s.n_elements * eb > 0xFFFFFF00ull) return fail(RS_EINVAL, "stream %u exceeds the 4 GiB addressing limit", i);
        if (s.n_parents && !s.offsets) return fail(RS_EINVAL, "stream %u: offsets is NULL", i);
        if (s.n_elements && !s.elements) return fail(RS_EINVAL, "stream %u: elements is NULL", i);
        if (s.n_parents && text != (s.lengths != nullptr))
            return fail(RS_EINVAL, text ? "stream %u: text streams need starts + lengths" : "stream %u: u32 streams need CSR offsets", i);
        if (d->kind == RS_GRAPH_THRESH && s.n_parents && !s.parent_param)
            return fail(RS_EINVAL, "stream %u: RS_GRAPH_THRESH needs parent_param", i);
        if ((uintptr_t)s.elements & 15u) return fail(RS_EINVAL, "stream %u: element array must be 16-byte aligned", i);
        const rs_agg_view &o = out[i];
        if (s.n_parents && (((d->agg_fields & RS_COUNT) && !o.count) || ((d->agg_fields & RS_SUM) && !o.sum) ||
                            ((d->agg_fields & RS_MIN) && !o.min) || ((d->agg_fields & RS_MAX) && !o.max) ||
                            ((d->agg_fields & RS_KEPT_COUNT) && !o.kept_count) ||
                            ((d->agg_fields & RS_KEPT_SUM) && !o.kept_sum)))
            return fail(RS_EINVAL, "stream %u: a destination of a requested field is NULL", i);
        uint32_t B = 1, nc = 0;
        const uint32_t P = (uint32_t)s.n_parents;
        claim_plan(d->kind, false, d->ensemble_width, P, P ? (double)s.n_elements / P : 0.0, &B, &nc);
        rs::StreamDev &e = tab.s[i];
        e.elements = s.elements;
        e.offsets = s.offsets;
        e.lengths = s.lengths;
        e.pparam = s.parent_param;
        e.agg_count = o.count;
        e.agg_sum = (unsigned long long *)o.sum;
        e.agg_min = o.min;
        e.agg_max = o.max;
        e.agg_kcount = o.kept_count;
        e.agg_ksum = (unsigned long long *)o.kept_sum;
        e.n_parents = P;
        e.n_elements = (uint32_t)s.n_elements;
        e.parents_per_claim = B;
        e.n_claims = nc;
        e.claim_begin = (uint32_t)claims;
        claims += nc;
        bmax = std::max(bmax, std::min(B, P));
    }
    if (claims >= (1ull << 32) - (1ull << 20)) return fail(RS_EINVAL, "too many claims in one call");
    // ---- device state: the scratch array of the current device (no allocation)
    void *base = nullptr;
    int hrc = rs::noalloc_scratch(&base);
    if (hrc) return fail(RS_EDEVICE, "scratch lookup: %s", hipGetErrorString((hipError_t)hrc));
    for (uint32_t i = 0; i < n_streams; ++i)
        tab.s[i].stats = (unsigned long long *)((uint8_t *)base + rs::NOALLOC_STATS_OFF) + i * rs::ST_WORDS;
    int dev = 0, n_cu = 0;
    HIP_OR(hipGetDevice(&dev), RS_EDEVICE);
    HIP_OR(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev), RS_EDEVICE);
    const int per_cu = rs::blocks_per_cu(d->kind, d->strategy, d->ensemble_width, qdepth, bmax);
    if (per_cu <= 0) return fail(RS_EINVAL, "the queues do not fit a compute unit's LDS at this width and depth");
    rs::LaunchArgs a{};
    a.streams = (const rs::StreamDev *)((uint8_t *)base + rs::NOALLOC_TABLE_OFF);
    a.ctl = (uint32_t *)((uint8_t *)base + rs::NOALLOC_CTL_OFF);
    a.n_streams = n_streams;
    a.total_claims = (uint32_t)claims;
    std::memcpy(a.param, d->param, sizeof a.param);
    a.agg_fields = d->agg_fields;
    a.collect_stats = 0;
    a.emit_outputs = 0;
    a.bmax = bmax;
    a.n_parts = rs::CTL_NPART;
    a.lb_wait_us = lookback_wait_us();
    a.qdepth = qdepth;
    const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((claims + 1) / 2, (uint64_t)per_cu * n_cu));
    hrc = rs::launch_noalloc_init(base, tab, hip_stream);
    if (hrc) return fail(RS_EDEVICE, "init launch: %s", hipGetErrorString((hipError_t)hrc));
    if (claims) {
        hrc = rs::launch_pipeline(d->kind, d->strategy, d->ensemble_width, a, grid, hip_stream);
        if (hrc) return fail(RS_EDEVICE, "kernel launch failed: %s", hipGetErrorString((hipError_t)hrc));
    }
    if (flags & RS_RUN_ASYNC) return RS_OK;
    // ---- synchronous call: the device's verdict
    HIP_OR(hipStreamSynchronize((hipStream_t)hip_stream), RS_EDEVICE);
    uint32_t err = 0;
    HIP_OR(hipMemcpy(&err, (uint8_t *)base + rs::NOALLOC_CTL_OFF + 4 * rs::CTL_ERROR, 4, hipMemcpyDeviceToHost), RS_EDEVICE);
    if (err) return fail(RS_EDEVICE, "the device scheduler stopped a claim (watchdog or internal check)");
    for (uint32_t i = 0; i < n_streams; ++i) {
        uint32_t bad = 0;
        HIP_OR(hipMemcpy(&bad, tab.s[i].stats + rs::ST_ERROR, 4, hipMemcpyDeviceToHost), RS_EDEVICE);
        if (bad) return fail(RS_EINVAL, "stream %u has malformed regions (out of order or past n_elements)", i);
    }
    return RS_OK;
}

RS_API int hbm_probe(const void *src, void *dst, uint64_t bytes, void *hip_stream) {
    clear_error();
    if (!src || !dst) return fail(RS_EINVAL, "NULL argument");
    if (((uintptr_t)src | (uintptr_t)dst | bytes) & 15u) return fail(RS_EINVAL, "pointers and size must be 16-byte multiples");
    int dev = 0;
    HIP_OR(hipGetDevice(&dev), RS_EDEVICE);
    hipDeviceProp_t prop;
    HIP_OR(hipGetDeviceProperties(&prop, dev), RS_EDEVICE);
    const int rc = rs::launch_probe_copy(src, dst, bytes, (uint32_t)prop.multiProcessorCount, hip_stream);
    if (rc) return fail(RS_EDEVICE, "probe launch: %s", hipGetErrorString((hipError_t)rc));
    return RS_OK;
}

RS_API int kernel_times(rs_pipeline *p, float *ms, uint32_t cap, uint32_t *n) {
    clear_error();
    if (!p || !n) return fail(RS_EINVAL, "NULL argument");
    if (!(p->d.flags & RS_TIME_KERNEL)) return fail(RS_EINVAL, "the pipeline was created without RS_TIME_KERNEL");
    if (cap && !ms) return fail(RS_EINVAL, "NULL ms with cap > 0");
    uint32_t k = 0;
    while (!p->timed.empty()) {
        const auto ev = p->timed.front();
        float t = 0.f;
        HIP_OR(hipEventSynchronize(ev.second), RS_EDEVICE);
        HIP_OR(hipEventElapsedTime(&t, ev.first, ev.second), RS_EDEVICE);
        p->timed.pop_front();
        p->spare_events.push_back(ev);
        if (k < cap) ms[k] = t;
        ++k;
    }
    *n = k;
    return RS_OK;
}

RS_API int pipeline_destroy(rs_pipeline *p) {
    if (!p) return RS_OK;
    if (p->user_stream) (void)hipStreamSynchronize(p->user_stream);
    for (auto &h : p->own)
        if (h) (void)hipStreamSynchronize(h);
    for (auto *q : {&p->timed, &p->spare_events})
        for (auto &ev : *q) {
            (void)hipEventDestroy(ev.first);
            (void)hipEventDestroy(ev.second);
        }
    if (p->copy) (void)hipStreamSynchronize(p->copy);
    p->batches.clear();
    p->streams.clear();
    for (auto &h : p->own)
        if (h) (void)hipStreamDestroy(h);
    if (p->copy) (void)hipStreamDestroy(p->copy);
    delete p;
    bool last = false;
    {
        std::lock_guard<std::mutex> g(g_live_mu);
        last = --g_live_pipelines == 0;
    }
    if (last) block_cache().trim();   // nothing can use a cached block any more
    return RS_OK;
}
