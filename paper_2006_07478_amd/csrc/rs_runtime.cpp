// Host runtime behind the C ABI (include/regionstream.h).
//
// A pipeline owns a HIP stream, a small device control block that the persistent
// kernel returns to zero on exit, and the device state of its streams.  run()
// gathers every pushed stream that fits the HBM budget into one work table and
// launches the persistent kernel once for all of them (§2.2: processors compete
// for a common input through atomics and the kernel returns only when the input
// is consumed).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/regionstream.h"
#include "rs_internal.h"

#define RS_API extern "C" __attribute__((visibility("default")))

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OR(expr, code)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) return fail(code, "%s: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

uint32_t k_max_of(uint32_t kind) { return kind == RS_HASH_EXPAND ? 3u : 1u; }
uint32_t elem_bytes_of(uint32_t kind) { return kind == RS_TEXT_WORDS ? 1u : 4u; }

enum StreamState { S_PUSHED = 0, S_LAUNCHED = 1, S_DONE = 2 };

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    int alloc(size_t bytes) {
        if (bytes == 0) bytes = 16;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(RS_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
        }
        return RS_OK;
    }
};

struct Stream {
    uint64_t id = 0;
    StreamState state = S_PUSHED;
    uint32_t n_parents = 0, n_elements = 0;
    const void *elements = nullptr;
    const uint32_t *offsets = nullptr, *lengths = nullptr, *pparam = nullptr;
    DevBuf own_elements, own_offsets, own_lengths, own_pparam;
    DevBuf count, sum, min, max, stats;
    uint32_t B = 1, n_claims = 0;
    uint64_t footprint = 0;
    uint64_t batch = 0;            // launch batch this stream ran in
    std::shared_ptr<hipEvent_t> done;
};

struct Batch {
    std::vector<uint64_t> ids;
    DevBuf table;
    uint32_t total_claims = 0;
    uint32_t grid = 0;
    rs::LaunchArgs args{};
    hipGraphExec_t graph = nullptr;
    ~Batch() {
        if (graph) (void)hipGraphExecDestroy(graph);
    }
};

}  // namespace

struct rs_pipeline {
    rs_pipeline_desc d{};
    int device = 0;
    int n_cu = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    DevBuf ctl, dummy;
    uint32_t width = 0, strategy = 0;
    uint64_t next_id = 1, next_batch = 1;
    uint64_t admitted_bytes = 0;
    std::map<uint64_t, std::unique_ptr<Stream>> streams;
    std::map<uint64_t, std::unique_ptr<Batch>> batches;
    uint64_t last_batch = 0;
};

namespace {

// Pick ensemble width and strategy for a pipeline whose description left them open,
// from the mean region length of the first stream (the paper's §5 observation: the
// right mechanism depends on elements per region relative to the SIMD width).
void resolve_config(rs_pipeline *p, double mean_len) {
    if (p->d.ensemble_width) p->width = p->d.ensemble_width;
    if (p->d.strategy != RS_AUTO) p->strategy = p->d.strategy;
    if (!p->width) p->width = 256;
    if (p->d.strategy == RS_AUTO && !p->strategy) p->strategy = mean_len >= 2.0 * p->width ? RS_SIGNAL : RS_TAG;
}

int check_stream(const rs_pipeline *p, const rs_stream_desc *s) {
    if (!s) return fail(RS_EINVAL, "stream description is NULL");
    if (s->mem != RS_MEM_HOST && s->mem != RS_MEM_DEVICE) return fail(RS_EINVAL, "mem must be RS_MEM_HOST or RS_MEM_DEVICE");
    const uint32_t eb = elem_bytes_of(p->d.kind);
    if (s->elem_bytes != eb) return fail(RS_EINVAL, "elem_bytes must be %u for this kind", eb);
    if (s->n_parents >= (1ull << 32)) return fail(RS_EINVAL, "n_parents must be < 2^32");
    if (s->n_elements * eb > 0xFFFFFF00ull) return fail(RS_EINVAL, "stream of %llu bytes exceeds the 4 GiB addressing limit",
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
                if (st < prev_end) return fail(RS_EINVAL, "region %llu starts before the previous one ends", (unsigned long long)i);
                if (en > s->n_elements) return fail(RS_EINVAL, "region %llu ends past n_elements", (unsigned long long)i);
                prev_end = en;
            }
        }
    }
    return RS_OK;
}

}  // namespace

// ------------------------------------------------------------------------------ ABI

RS_API const char *rs_last_error(void) { return g_err.c_str(); }

RS_API int pipeline_create(const rs_pipeline_desc *d, rs_pipeline **out) {
    g_err.clear();
    if (!d || !out) return fail(RS_EINVAL, "NULL argument");
    *out = nullptr;
    if (d->abi_version != RS_ABI_VERSION) return fail(RS_EINVAL, "abi_version %u, library is %u", d->abi_version, RS_ABI_VERSION);
    if (d->kind < RS_MODFILTER || d->kind > RS_GRAPH_THRESH) return fail(RS_EINVAL, "unknown kind %u", d->kind);
    if (d->strategy > RS_AUTO) return fail(RS_EINVAL, "unknown strategy %u", d->strategy);
    if (d->agg_fields == 0 || (d->agg_fields & ~15u)) return fail(RS_EINVAL, "agg_fields must be a non-empty OR of RS_COUNT|RS_SUM|RS_MIN|RS_MAX");
    const uint32_t w = d->ensemble_width;
    if (w && !rs::kernel_supported(d->kind, RS_TAG, w))
        return fail(RS_EINVAL, "ensemble_width %u not supported (64, 128, 256 or 512)", w);
    if (d->queue_depth) {
        const uint32_t q = d->queue_depth;
        if (q & (q - 1)) return fail(RS_EINVAL, "queue_depth must be a power of two");
        if (w && q < 2 * w) return fail(RS_EINVAL, "queue_depth %u < 2 * ensemble_width", q);
    }
    if (d->emit_outputs > 1) return fail(RS_EINVAL, "emit_outputs must be 0 or 1");
    if (d->emit_outputs) return fail(RS_EINVAL, "the ordered output stream is not available in this build");
    if (d->kind == RS_MODFILTER && d->param[0] != 0 && d->param[1] >= d->param[0])
        return fail(RS_EINVAL, "residue must be smaller than the modulus");

    std::unique_ptr<rs_pipeline> p(new rs_pipeline);
    p->d = *d;
    HIP_OR(hipGetDevice(&p->device), RS_EDEVICE);
    hipDeviceProp_t prop;
    HIP_OR(hipGetDeviceProperties(&prop, p->device), RS_EDEVICE);
    p->n_cu = prop.multiProcessorCount;
    HIP_OR(hipStreamCreateWithFlags(&p->own_stream, hipStreamNonBlocking), RS_EDEVICE);
    p->stream = p->own_stream;
    int rc = p->ctl.alloc(rs::CTL_WORDS * sizeof(uint32_t));
    if (rc) return rc;
    rc = p->dummy.alloc(256);
    if (rc) return rc;
    HIP_OR(hipMemset(p->ctl.p, 0, rs::CTL_WORDS * sizeof(uint32_t)), RS_EDEVICE);
    HIP_OR(hipMemset(p->dummy.p, 0, 256), RS_EDEVICE);
    if (d->ensemble_width) p->width = d->ensemble_width;
    if (d->strategy != RS_AUTO) p->strategy = d->strategy;
    *out = p.release();
    return RS_OK;
}

RS_API int pipeline_set_stream(rs_pipeline *p, void *hip_stream) {
    if (!p) return fail(RS_EINVAL, "NULL pipeline");
    p->stream = hip_stream ? (hipStream_t)hip_stream : p->own_stream;
    return RS_OK;
}

RS_API int stream_push(rs_pipeline *p, const rs_stream_desc *s, uint64_t *stream_id) {
    g_err.clear();
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

    // mean region length picks the claim size and, if open, the configuration
    double covered = 0;
    if (s->mem == RS_MEM_HOST && P) {
        if (lens) {
            for (uint64_t i = 0; i < P; ++i) covered += lens[i];
        } else {
            covered = (double)offs[P] - (double)offs[0];
        }
    } else {
        covered = (double)s->n_elements;
    }
    const double mean_len = P ? covered / (double)P : 0.0;
    if (!p->width || (p->d.strategy == RS_AUTO && !p->strategy)) resolve_config(p, mean_len);
    const uint32_t bmax = rs::claim_parents_max(p->width);
    const double target = 16.0 * p->width;
    double b = mean_len > 0 ? target / mean_len : (double)bmax;
    st->B = (uint32_t)std::max(1.0, std::min((double)bmax, b));
    st->n_claims = (uint32_t)((P + st->B - 1) / st->B);

    // footprint on the device
    const uint64_t agg_bytes = P * ((p->d.agg_fields & RS_COUNT ? 4 : 0) + (p->d.agg_fields & RS_SUM ? 8 : 0) +
                                    (p->d.agg_fields & RS_MIN ? 4 : 0) + (p->d.agg_fields & RS_MAX ? 4 : 0));
    uint64_t in_bytes = 0;
    if (s->mem == RS_MEM_HOST)
        in_bytes = s->n_elements * eb + (lens ? 8 * P : 4 * (P + 1)) + (s->parent_param ? 4 * P : 0);
    st->footprint = in_bytes + agg_bytes + 8 * rs::ST_WORDS;
    if (p->d.hbm_budget_bytes && st->footprint > p->d.hbm_budget_bytes)
        return fail(RS_EBUDGET, "stream needs %llu bytes, budget is %llu", (unsigned long long)st->footprint,
                    (unsigned long long)p->d.hbm_budget_bytes);

    hipStream_t hs = p->stream;
    if (s->mem == RS_MEM_HOST) {
        if ((rc = st->own_elements.alloc(s->n_elements * eb + 16))) return rc;
        if (s->n_elements)
            HIP_OR(hipMemcpyAsync(st->own_elements.p, s->elements, s->n_elements * eb, hipMemcpyHostToDevice, hs), RS_EDEVICE);
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
        // the host arrays may be reused by the caller as soon as we return
        HIP_OR(hipStreamSynchronize(hs), RS_EDEVICE);
    } else {
        st->elements = s->elements;
        st->offsets = s->offsets;
        st->lengths = s->lengths;
        st->pparam = s->parent_param;
        if (P) {
            rc = rs::validate_device_regions(st->offsets, st->lengths, (uint32_t)P, st->n_elements, hs);
            if (rc > 0) return fail(RS_EINVAL, "device regions are malformed (first bad parent %d)", rc - 1);
            if (rc < 0) return fail(RS_EDEVICE, "region validation failed: %s", hipGetErrorString((hipError_t)-rc));
        }
    }
    if (p->d.agg_fields & RS_COUNT && (rc = st->count.alloc(4 * P))) return rc;
    if (p->d.agg_fields & RS_SUM && (rc = st->sum.alloc(8 * P))) return rc;
    if (p->d.agg_fields & RS_MIN && (rc = st->min.alloc(4 * P))) return rc;
    if (p->d.agg_fields & RS_MAX && (rc = st->max.alloc(4 * P))) return rc;
    if ((rc = st->stats.alloc(8 * rs::ST_WORDS))) return rc;
    HIP_OR(hipMemset(st->stats.p, 0, 8 * rs::ST_WORDS), RS_EDEVICE);

    st->id = p->next_id++;
    *stream_id = st->id;
    p->streams[st->id] = std::move(st);
    return RS_OK;
}

namespace {

int launch_batch(rs_pipeline *p, Batch &b) {
    const int rc = rs::launch_pipeline(p->d.kind, p->strategy, p->width, b.args, b.grid, p->stream);
    if (rc) return fail(RS_EDEVICE, "kernel launch failed: %s", hipGetErrorString((hipError_t)rc));
    return RS_OK;
}

int make_batch(rs_pipeline *p, const std::vector<Stream *> &sel, std::unique_ptr<Batch> &out) {
    std::unique_ptr<Batch> b(new Batch);
    std::vector<rs::StreamDev> h(sel.size());
    uint32_t claims = 0;
    for (size_t i = 0; i < sel.size(); ++i) {
        Stream *s = sel[i];
        rs::StreamDev &e = h[i];
        std::memset(&e, 0, sizeof e);
        e.elements = s->elements;
        e.offsets = s->offsets;
        e.lengths = s->lengths;
        e.pparam = s->pparam;
        e.agg_count = (uint32_t *)s->count.p;
        e.agg_sum = (unsigned long long *)s->sum.p;
        e.agg_min = (uint32_t *)s->min.p;
        e.agg_max = (uint32_t *)s->max.p;
        e.stats = (unsigned long long *)s->stats.p;
        e.n_parents = s->n_parents;
        e.n_elements = s->n_elements;
        e.parents_per_claim = s->B;
        e.n_claims = s->n_claims;
        e.claim_begin = claims;
        claims += s->n_claims;
        b->ids.push_back(s->id);
    }
    int rc = b->table.alloc(sizeof(rs::StreamDev) * std::max<size_t>(1, h.size()));
    if (rc) return rc;
    HIP_OR(hipMemcpyAsync(b->table.p, h.data(), sizeof(rs::StreamDev) * h.size(), hipMemcpyHostToDevice, p->stream),
           RS_EDEVICE);
    HIP_OR(hipStreamSynchronize(p->stream), RS_EDEVICE);   // h is a local array
    b->total_claims = claims;
    const int per_cu = rs::blocks_per_cu(p->d.kind, p->strategy, p->width);
    if (per_cu <= 0) return fail(RS_EDEVICE, "kernel does not fit on a compute unit");
    b->grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(claims, (uint64_t)per_cu * p->n_cu));
    rs::LaunchArgs &a = b->args;
    a.streams = (const rs::StreamDev *)b->table.p;
    a.ctl = (uint32_t *)p->ctl.p;
    a.dummy = p->dummy.p;
    a.n_streams = (uint32_t)sel.size();
    a.total_claims = claims;
    std::memcpy(a.param, p->d.param, sizeof a.param);
    a.agg_fields = p->d.agg_fields;
    a.collect_stats = (p->d.flags & RS_COLLECT_STATS) ? 1u : 0u;
    a.emit_outputs = p->d.emit_outputs;
    out = std::move(b);
    return RS_OK;
}

int finish_check(rs_pipeline *p) {
    uint32_t err = 0;
    HIP_OR(hipMemcpy(&err, (uint32_t *)p->ctl.p + rs::CTL_ERROR, 4, hipMemcpyDeviceToHost), RS_EDEVICE);
    if (err) {
        const uint32_t zero = 0;
        (void)hipMemcpy((uint32_t *)p->ctl.p + rs::CTL_ERROR, &zero, 4, hipMemcpyHostToDevice);
        return fail(RS_EDEVICE, "the device scheduler stopped a claim (watchdog or internal check)");
    }
    return RS_OK;
}

}  // namespace

RS_API int run(rs_pipeline *p, uint32_t flags) {
    g_err.clear();
    if (!p) return fail(RS_EINVAL, "NULL pipeline");
    if (flags & ~7u) return fail(RS_EINVAL, "unknown run flags");
    std::vector<Stream *> sel;
    uint64_t budget_used = p->admitted_bytes;
    for (auto &kv : p->streams) {
        Stream *s = kv.second.get();
        if (s->state != S_PUSHED) continue;
        if (p->d.hbm_budget_bytes && budget_used + s->footprint > p->d.hbm_budget_bytes) continue;
        budget_used += s->footprint;
        sel.push_back(s);
    }
    if (sel.empty()) return RS_OK;
    if (!p->width) resolve_config(p, 0.0);

    std::vector<std::vector<Stream *>> groups;
    if (flags & RS_RUN_PER_STREAM) {
        for (Stream *s : sel) groups.push_back({s});
    } else {
        groups.push_back(sel);
    }
    for (auto &grp : groups) {
        std::unique_ptr<Batch> b;
        int rc = make_batch(p, grp, b);
        if (rc) return rc;
        if (b->total_claims) {
            rc = launch_batch(p, *b);
            if (rc) return rc;
        }
        auto ev = std::shared_ptr<hipEvent_t>(new hipEvent_t(nullptr), [](hipEvent_t *e) {
            if (*e) (void)hipEventDestroy(*e);
            delete e;
        });
        HIP_OR(hipEventCreateWithFlags(ev.get(), hipEventDisableTiming), RS_EDEVICE);
        HIP_OR(hipEventRecord(*ev, p->stream), RS_EDEVICE);
        const uint64_t bid = p->next_batch++;
        for (Stream *s : grp) {
            s->state = S_LAUNCHED;
            s->done = ev;
            s->batch = bid;
            p->admitted_bytes += s->footprint;
        }
        p->batches[bid] = std::move(b);
        p->last_batch = bid;
    }
    if (!(flags & RS_RUN_ASYNC)) {
        HIP_OR(hipStreamSynchronize(p->stream), RS_EDEVICE);
        return finish_check(p);
    }
    return RS_OK;
}

// Re-run the most recent batch in place (benchmarks and graph replay).  The launch is
// captured into a HIP graph on first use unless RS_NO_GRAPH or statistics are enabled.
RS_API int run_again(rs_pipeline *p, uint32_t flags) {
    g_err.clear();
    if (!p) return fail(RS_EINVAL, "NULL pipeline");
    auto it = p->batches.find(p->last_batch);
    if (it == p->batches.end()) return fail(RS_ESTATE, "no batch has run on this pipeline");
    Batch &b = *it->second;
    if (b.total_claims) {
        const bool use_graph = !(p->d.flags & (RS_NO_GRAPH | RS_COLLECT_STATS));
        if (use_graph) {
            if (!b.graph) {
                hipGraph_t g = nullptr;
                HIP_OR(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal), RS_EDEVICE);
                const int rc = rs::launch_pipeline(p->d.kind, p->strategy, p->width, b.args, b.grid, p->stream);
                hipError_t e = hipStreamEndCapture(p->stream, &g);
                if (rc || e != hipSuccess) return fail(RS_EDEVICE, "graph capture failed");
                e = hipGraphInstantiate(&b.graph, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e != hipSuccess) return fail(RS_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
            }
            HIP_OR(hipGraphLaunch(b.graph, p->stream), RS_EDEVICE);
        } else {
            int rc = launch_batch(p, b);
            if (rc) return rc;
        }
    }
    if (!(flags & RS_RUN_ASYNC)) {
        HIP_OR(hipStreamSynchronize(p->stream), RS_EDEVICE);
        return finish_check(p);
    }
    return RS_OK;
}

namespace {

int find_done(rs_pipeline *p, uint64_t id, uint32_t flags, Stream **out) {
    auto it = p->streams.find(id);
    if (it == p->streams.end()) return fail(RS_ENOTFOUND, "unknown stream id %llu", (unsigned long long)id);
    Stream *s = it->second.get();
    if (s->state == S_PUSHED) return fail(RS_ESTATE, "stream %llu has not been run", (unsigned long long)id);
    if (s->state == S_LAUNCHED) {
        if (flags & RS_NONBLOCK) {
            hipError_t e = hipEventQuery(*s->done);
            if (e == hipErrorNotReady) return fail(RS_ENOTREADY, "stream %llu is still running", (unsigned long long)id);
            if (e != hipSuccess) return fail(RS_EDEVICE, "hipEventQuery: %s", hipGetErrorString(e));
        } else {
            HIP_OR(hipEventSynchronize(*s->done), RS_EDEVICE);
        }
        int rc = finish_check(p);
        if (rc) return rc;
        s->state = S_DONE;
    }
    *out = s;
    return RS_OK;
}

void release(rs_pipeline *p, Stream *s) {
    p->admitted_bytes -= std::min(p->admitted_bytes, s->footprint);
    p->streams.erase(s->id);
}

}  // namespace

RS_API int read_aggregates(rs_pipeline *p, uint64_t stream_id, rs_agg_view *out, uint32_t flags) {
    g_err.clear();
    if (!p || !out) return fail(RS_EINVAL, "NULL argument");
    Stream *s = nullptr;
    int rc = find_done(p, stream_id, flags, &s);
    if (rc) return rc;
    const hipMemcpyKind k = (flags & RS_READ_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const size_t P = s->n_parents;
    struct F { void *dst; DevBuf *src; size_t bytes; uint32_t bit; const char *name; };
    F fields[4] = {{out->count, &s->count, 4 * P, RS_COUNT, "count"},
                   {out->sum, &s->sum, 8 * P, RS_SUM, "sum"},
                   {out->min, &s->min, 4 * P, RS_MIN, "min"},
                   {out->max, &s->max, 4 * P, RS_MAX, "max"}};
    for (auto &f : fields) {
        if (!f.dst) continue;
        if (!(p->d.agg_fields & f.bit)) return fail(RS_EINVAL, "field %s is not stored by this pipeline", f.name);
        if (P) HIP_OR(hipMemcpy(f.dst, f.src->p, f.bytes, k), RS_EDEVICE);
    }
    if (flags & RS_READ_RELEASE) release(p, s);
    return RS_OK;
}

RS_API int read_outputs(rs_pipeline *p, uint64_t stream_id, uint32_t *out, uint64_t cap, uint64_t *n_out, uint32_t flags) {
    g_err.clear();
    if (!p) return fail(RS_EINVAL, "NULL pipeline");
    (void)stream_id; (void)out; (void)cap; (void)n_out; (void)flags;
    return fail(RS_EINVAL, "pipeline was created without emit_outputs");
}

RS_API int rs_stats(rs_pipeline *p, uint64_t stream_id, rs_stats_t *out) {
    g_err.clear();
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
    out->n_outputs = st[rs::ST_OUTPUTS];
    out->ensemble_width = p->width;
    out->queue_depth = 2 * p->width;
    out->strategy = p->strategy;
    auto bi = p->batches.find(s->batch);
    out->n_workgroups = bi != p->batches.end() ? bi->second->grid : 0;
    return RS_OK;
}

RS_API int stream_release(rs_pipeline *p, uint64_t stream_id) {
    g_err.clear();
    if (!p) return fail(RS_EINVAL, "NULL pipeline");
    auto it = p->streams.find(stream_id);
    if (it == p->streams.end()) return fail(RS_ENOTFOUND, "unknown stream id %llu", (unsigned long long)stream_id);
    Stream *s = it->second.get();
    if (s->state == S_LAUNCHED) {
        if (hipEventQuery(*s->done) == hipErrorNotReady) return fail(RS_ESTATE, "stream is still running");
        s->state = S_DONE;
    }
    release(p, s);
    return RS_OK;
}

RS_API int pipeline_destroy(rs_pipeline *p) {
    if (!p) return RS_OK;
    (void)hipStreamSynchronize(p->stream);
    (void)hipStreamSynchronize(p->own_stream);
    p->streams.clear();
    p->batches.clear();
    if (p->own_stream) (void)hipStreamDestroy(p->own_stream);
    delete p;
    return RS_OK;
}
