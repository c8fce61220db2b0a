// Drives the host runtime through the C ABI for a build whose host code carries AddressSanitizer
// and UndefinedBehaviorSanitizer.  "cpu" runs the paths that need no device: every refusal of a
// description, a stream or an argument, and the error messages.  "gpu" also runs the bookkeeping
// paths on a device: streams pushed from host memory, batched and one-launch-per-stream runs,
// reads, releases, a malformed stream, the serving loop and the no-allocation entry point; their
// results are checked against each other (parity with the oracle is the other tests' job).
// Exit status 0 when every check held; each failure prints its line and the library's message.
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "regionstream.h"

static int g_fails = 0;
#define EXPECT(c)                                                                                   \
    do {                                                                                            \
        if (!(c)) {                                                                                 \
            std::fprintf(stderr, "FAIL line %d: %s (last error: %s)\n", __LINE__, #c, rs_last_error()); \
            ++g_fails;                                                                              \
        }                                                                                           \
    } while (0)

static rs_pipeline_desc desc(uint32_t kind, uint32_t strategy, uint32_t width) {
    rs_pipeline_desc d;
    std::memset(&d, 0, sizeof d);
    d.abi_version = RS_ABI_VERSION;
    d.kind = kind;
    d.strategy = strategy;
    d.agg_fields = RS_COUNT | RS_SUM;
    d.ensemble_width = width;
    return d;
}

// Descriptions every build must refuse before touching a device.
static void refused_descriptions() {
    std::vector<rs_pipeline_desc> bad;
    rs_pipeline_desc d = desc(RS_HASH_EXPAND, RS_TAG, 256);
    d.abi_version = 999; bad.push_back(d);
    d = desc(0, RS_TAG, 256); bad.push_back(d);
    d = desc(6, RS_TAG, 256); bad.push_back(d);
    d = desc(RS_HASH_EXPAND, 9, 256); bad.push_back(d);
    d = desc(RS_HASH_EXPAND, RS_TAG, 256); d.agg_fields = 0; bad.push_back(d);
    d = desc(RS_HASH_EXPAND, RS_TAG, 256); d.agg_fields = RS_KEPT_COUNT; bad.push_back(d);
    d = desc(RS_HASH_TREE, RS_TAG, 256); d.agg_fields = 64; bad.push_back(d);
    d = desc(RS_HASH_EXPAND, RS_TAG, 100); bad.push_back(d);
    d = desc(RS_HASH_EXPAND, RS_TAG, 2048); bad.push_back(d);
    d = desc(RS_HASH_EXPAND, RS_TAG, 256); d.queue_depth = 4096; bad.push_back(d);
    d = desc(RS_HASH_EXPAND, RS_TAG, 256); d.queue_depth = 768; bad.push_back(d);
    d = desc(RS_HASH_EXPAND, RS_TAG, 256); d.queue_depth = 256; bad.push_back(d);
    d = desc(RS_MODFILTER, RS_TAG, 64); d.param[0] = 4; d.param[1] = 4; bad.push_back(d);
    d = desc(RS_MODFILTER, RS_ENUM_TAG, 64); bad.push_back(d);
    d = desc(RS_HASH_EXPAND, RS_SIGNAL_LANES, 1024); bad.push_back(d);
    d = desc(RS_TEXT_WORDS, RS_SIGNAL_LANES, 128); bad.push_back(d);
    for (size_t i = 0; i < bad.size(); ++i) {
        rs_pipeline *p = nullptr;
        const int rc = pipeline_create(&bad[i], &p);
        if (rc != RS_EINVAL || p != nullptr) std::fprintf(stderr, "  description %zu\n", i);
        EXPECT(rc == RS_EINVAL);
        EXPECT(p == nullptr);
        EXPECT(std::strlen(rs_last_error()) > 0);
    }
}

static void null_arguments() {
    rs_pipeline_desc d = desc(RS_HASH_EXPAND, RS_TAG, 256);
    rs_pipeline *p = nullptr;
    uint64_t id = 0;
    rs_stream_desc s;
    std::memset(&s, 0, sizeof s);
    rs_agg_view v;
    std::memset(&v, 0, sizeof v);
    rs_stats_t st;
    uint32_t u = 0;
    uint64_t n = 0;
    float ms = 0;
    rs_request_timing tim;
    EXPECT(pipeline_create(nullptr, &p) == RS_EINVAL);
    EXPECT(pipeline_create(&d, nullptr) == RS_EINVAL);
    EXPECT(stream_push(nullptr, &s, &id) == RS_EINVAL);
    EXPECT(run(nullptr, 0) == RS_EINVAL);
    EXPECT(run_again(nullptr, 0) == RS_EINVAL);
    EXPECT(read_aggregates(nullptr, 1, &v, 0) == RS_EINVAL);
    EXPECT(read_outputs(nullptr, 1, &u, 1, &n, 0) == RS_EINVAL);
    EXPECT(rs_stats(nullptr, 1, &st) == RS_EINVAL);
    EXPECT(kernel_times(nullptr, &ms, 1, &u) == RS_EINVAL);
    EXPECT(stream_release(nullptr, 1) != RS_OK);
    EXPECT(serve(nullptr, nullptr, 0, nullptr, &tim, 0) == RS_EINVAL);
    EXPECT(pipeline_set_stream(nullptr, nullptr) == RS_EINVAL);
    EXPECT(run_noalloc(nullptr, &s, 1, &v, nullptr, 0) == RS_EINVAL);
    EXPECT(run_noalloc(&d, nullptr, 1, &v, nullptr, 0) == RS_EINVAL);
}

// run_noalloc checks everything on the host before it touches the device.
static void noalloc_refusals() {
    static uint32_t elems[64] __attribute__((aligned(16)));
    static uint32_t offs[2] = {0, 64};
    uint32_t cnt[1];
    uint64_t sum[1];
    rs_agg_view v;
    std::memset(&v, 0, sizeof v);
    v.count = cnt;
    v.sum = sum;
    rs_stream_desc s;
    std::memset(&s, 0, sizeof s);
    s.mem = RS_MEM_DEVICE;
    s.elem_bytes = 4;
    s.n_parents = 1;
    s.n_elements = 64;
    s.offsets = offs;
    s.elements = elems;
    rs_pipeline_desc d = desc(RS_HASH_EXPAND, RS_TAG, 256);
    std::vector<rs_stream_desc> many(17, s);
    std::vector<rs_agg_view> outs(17, v);
    EXPECT(run_noalloc(&d, many.data(), 0, outs.data(), nullptr, 0) == RS_EINVAL);
    EXPECT(run_noalloc(&d, many.data(), 17, outs.data(), nullptr, 0) == RS_EINVAL);
    rs_pipeline_desc a = d;
    a.strategy = RS_AUTO;
    EXPECT(run_noalloc(&a, &s, 1, &v, nullptr, 0) == RS_EINVAL);
    a = d;
    a.emit_outputs = 1;
    EXPECT(run_noalloc(&a, &s, 1, &v, nullptr, 0) == RS_EINVAL);
    a = d;
    a.agg_fields = RS_COUNT | RS_MIN;   // min has no destination
    EXPECT(run_noalloc(&a, &s, 1, &v, nullptr, 0) == RS_EINVAL);
    rs_stream_desc b = s;
    b.mem = RS_MEM_HOST;
    EXPECT(run_noalloc(&d, &b, 1, &v, nullptr, 0) == RS_EINVAL);
    b = s;
    b.elem_bytes = 1;
    EXPECT(run_noalloc(&d, &b, 1, &v, nullptr, 0) == RS_EINVAL);
    b = s;
    b.elements = (const uint8_t *)elems + 4;   // misaligned
    EXPECT(run_noalloc(&d, &b, 1, &v, nullptr, 0) == RS_EINVAL);
    b = s;
    b.offsets = nullptr;
    EXPECT(run_noalloc(&d, &b, 1, &v, nullptr, 0) == RS_EINVAL);
    b = s;
    b.n_elements = 1ull << 33;
    EXPECT(run_noalloc(&d, &b, 1, &v, nullptr, 0) == RS_EINVAL);
}

// ---- device paths ----

static uint32_t mix(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    return x;
}

struct HostStream {
    std::vector<uint32_t> offsets, elements;
};

static HostStream make_stream(uint32_t seed, uint32_t parents, uint32_t max_len) {
    HostStream h;
    h.offsets.push_back(0);
    for (uint32_t p = 0; p < parents; ++p) h.offsets.push_back(h.offsets.back() + mix(seed * 7919u + p) % (max_len + 1));
    h.elements.resize(h.offsets.back() + 1);
    for (uint32_t i = 0; i < h.elements.size(); ++i) h.elements[i] = mix(seed ^ (i * 2654435761u));
    h.elements.resize(h.offsets.back());
    return h;
}

static rs_stream_desc host_desc(const HostStream &h) {
    rs_stream_desc s;
    std::memset(&s, 0, sizeof s);
    s.mem = RS_MEM_HOST;
    s.elem_bytes = 4;
    s.n_parents = h.offsets.size() - 1;
    s.n_elements = h.elements.size();
    s.offsets = h.offsets.data();
    s.elements = h.elements.data();
    return s;
}

struct Agg {
    std::vector<uint32_t> count, min, max;
    std::vector<uint64_t> sum;
    explicit Agg(size_t P) : count(P + 1), min(P + 1), max(P + 1), sum(P + 1) {}
    rs_agg_view view() {
        rs_agg_view v;
        std::memset(&v, 0, sizeof v);
        v.count = count.data();
        v.sum = sum.data();
        v.min = min.data();
        v.max = max.data();
        return v;
    }
    bool operator==(const Agg &o) const { return count == o.count && sum == o.sum && min == o.min && max == o.max; }
};

static void device_paths() {
    std::vector<HostStream> hs;
    for (uint32_t i = 0; i < 6; ++i) hs.push_back(make_stream(i + 1, 50 + 400 * i, i % 2 ? 300 : 9));
    // batched run, then one launch per stream: equal records
    std::vector<Agg> batched, single;
    for (int per_stream = 0; per_stream < 2; ++per_stream) {
        rs_pipeline_desc d = desc(RS_HASH_EXPAND, RS_TAG, 128);
        d.agg_fields = RS_COUNT | RS_SUM | RS_MIN | RS_MAX;
        rs_pipeline *p = nullptr;
        EXPECT(pipeline_create(&d, &p) == RS_OK);
        if (!p) return;
        std::vector<uint64_t> ids;
        for (auto &h : hs) {
            rs_stream_desc s = host_desc(h);
            uint64_t id = 0;
            EXPECT(stream_push(p, &s, &id) == RS_OK);
            ids.push_back(id);
        }
        EXPECT(run(p, per_stream ? RS_RUN_PER_STREAM : 0) == RS_OK);
        for (size_t i = 0; i < hs.size(); ++i) {
            Agg a(hs[i].offsets.size() - 1);
            rs_agg_view v = a.view();
            EXPECT(read_aggregates(p, ids[i], &v, 0) == RS_OK);
            (per_stream ? single : batched).push_back(a);
        }
        rs_stats_t st;
        EXPECT(rs_stats(p, ids[0], &st) == RS_OK);
        for (uint64_t id : ids) EXPECT(stream_release(p, id) == RS_OK);
        EXPECT(stream_release(p, ids[0]) == RS_ENOTFOUND);
        // a host stream whose offsets decrease is refused at push
        HostStream bad = hs[0];
        std::swap(bad.offsets[1], bad.offsets[2]);
        if (bad.offsets[1] != bad.offsets[2]) {
            rs_stream_desc s = host_desc(bad);
            uint64_t id = 0;
            EXPECT(stream_push(p, &s, &id) == RS_EINVAL);
        }
        EXPECT(pipeline_destroy(p) == RS_OK);
    }
    for (size_t i = 0; i < hs.size(); ++i) EXPECT(batched[i] == single[i]);
    // the serving loop on the same streams: same records
    {
        rs_pipeline_desc d = desc(RS_HASH_EXPAND, RS_TAG, 128);
        d.agg_fields = RS_COUNT | RS_SUM | RS_MIN | RS_MAX;
        d.hbm_budget_bytes = 64 << 10;   // admission gates
        rs_pipeline *p = nullptr;
        EXPECT(pipeline_create(&d, &p) == RS_OK);
        if (!p) return;
        std::vector<rs_request> reqs(hs.size());
        std::vector<Agg> got;
        std::vector<rs_agg_view> views;
        std::vector<rs_request_timing> tim(hs.size());
        for (size_t i = 0; i < hs.size(); ++i) {
            reqs[i].arrival_s = 1e-4 * (double)i;
            reqs[i].stream = host_desc(hs[i]);
            got.emplace_back(hs[i].offsets.size() - 1);
        }
        for (auto &g : got) views.push_back(g.view());
        const int rc = serve(p, reqs.data(), reqs.size(), views.data(), tim.data(), 0);
        EXPECT(rc == RS_OK || rc == RS_EBUDGET);
        for (size_t i = 0; i < hs.size(); ++i)
            if (tim[i].status == RS_OK) EXPECT(got[i] == batched[i]);
        std::swap(reqs[0], reqs[1]);   // unsorted arrivals
        EXPECT(serve(p, reqs.data(), reqs.size(), views.data(), tim.data(), 0) == RS_EINVAL);
        EXPECT(pipeline_destroy(p) == RS_OK);
    }
    // the no-allocation entry point on device copies of two streams, twice
    {
        std::vector<void *> dev;
        std::vector<rs_stream_desc> ss;
        std::vector<Agg> got;
        for (int i = 0; i < 2; ++i) {
            const HostStream &h = hs[i + 1];
            void *o = nullptr, *e = nullptr;
            EXPECT(hipMalloc(&o, 4 * h.offsets.size()) == hipSuccess);
            EXPECT(hipMalloc(&e, 4 * h.elements.size() + 16) == hipSuccess);
            EXPECT(hipMemcpy(o, h.offsets.data(), 4 * h.offsets.size(), hipMemcpyHostToDevice) == hipSuccess);
            EXPECT(hipMemcpy(e, h.elements.data(), 4 * h.elements.size(), hipMemcpyHostToDevice) == hipSuccess);
            rs_stream_desc s = host_desc(h);
            s.mem = RS_MEM_DEVICE;
            s.offsets = (const uint32_t *)o;
            s.elements = e;
            ss.push_back(s);
            dev.push_back(o);
            dev.push_back(e);
        }
        std::vector<rs_agg_view> views;
        std::vector<void *> outs;
        for (int i = 0; i < 2; ++i) {
            const size_t P = hs[i + 1].offsets.size() - 1;
            rs_agg_view v;
            std::memset(&v, 0, sizeof v);
            EXPECT(hipMalloc((void **)&v.count, 4 * P) == hipSuccess);
            EXPECT(hipMalloc((void **)&v.sum, 8 * P) == hipSuccess);
            outs.push_back(v.count);
            outs.push_back(v.sum);
            views.push_back(v);
        }
        rs_pipeline_desc d = desc(RS_HASH_EXPAND, RS_SIGNAL, 128);
        for (int rep = 0; rep < 2; ++rep) {
            EXPECT(run_noalloc(&d, ss.data(), 2, views.data(), nullptr, 0) == RS_OK);
            for (int i = 0; i < 2; ++i) {
                const size_t P = hs[i + 1].offsets.size() - 1;
                std::vector<uint32_t> c(P);
                std::vector<uint64_t> s(P);
                EXPECT(hipMemcpy(c.data(), views[i].count, 4 * P, hipMemcpyDeviceToHost) == hipSuccess);
                EXPECT(hipMemcpy(s.data(), views[i].sum, 8 * P, hipMemcpyDeviceToHost) == hipSuccess);
                for (size_t q = 0; q < P; ++q) {
                    EXPECT(c[q] == batched[i + 1].count[q]);
                    EXPECT(s[q] == batched[i + 1].sum[q]);
                }
            }
        }
        for (void *q : dev) (void)hipFree(q);
        for (void *q : outs) (void)hipFree(q);
    }
}

int main(int argc, char **argv) {
    const bool gpu = argc > 1 && std::strcmp(argv[1], "gpu") == 0;
    refused_descriptions();
    null_arguments();
    noalloc_refusals();
    if (gpu) device_paths();
    std::printf("%s: %d failed checks\n", gpu ? "host and device paths" : "host paths", g_fails);
    return g_fails ? 1 : 0;
}
