/*
 * Seeded synthetic input generators shared by the oracle side and the GPU side.
 *
 * This file holds none of the method's arithmetic: it only draws inputs
 * (region sizes, element values, text bytes, degrees, weights, arrival times)
 * from counter-based random streams, so the same seed and index always give
 * the same value whatever the thread count.
 *
 * The random stream is SplitMix64's output function (Steele, Lea & Flood,
 * OOPSLA 2014): mix64(s + k * 0x9E3779B97F4A7C15) is the k-th output of the
 * generator seeded with s.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

static inline uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gen_mix64(uint64_t z) { return mix64(z); }

/* Uniform double in the open interval (0, 1) from 53 random bits. */
static inline double unit_open(uint64_t r) { return ((double)(r >> 11) + 0.5) * 0x1.0p-53; }

/* Geometric variate on {0, 1, ...} with success probability p (mean (1-p)/p). */
static inline uint64_t geometric(uint64_t r, double log1mp)
{
    double g = floor(log(unit_open(r)) / log1mp);
    if (g > 9.0e18) g = 9.0e18;
    return (uint64_t)g;
}

/* ---- Sum-app style regions: uniform sizes in [0, max_size] and u32 values ---- */

/* sizes[p] = mix64(mix64(seed ^ 0x5EED) + p) mod (max_size + 1). */
void gen_uniform_sizes(uint64_t seed, uint32_t max_size, uint64_t n_parents, uint32_t *sizes)
{
    uint64_t base = mix64(seed ^ 0x5EEDull);
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < (int64_t)n_parents; ++p)
        sizes[p] = (uint32_t)(mix64(base + (uint64_t)p) % ((uint64_t)max_size + 1u));
}

/* values of parent p, index i: (u32) mix64(mix64(seed) ^ (p << 32 | i)); offsets is CSR [P+1]. */
void gen_parent_values(uint64_t seed, uint64_t n_parents, const uint32_t *offsets, uint32_t *values)
{
    uint64_t base = mix64(seed);
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < (int64_t)n_parents; ++p)
        for (uint32_t e = offsets[p]; e < offsets[p + 1]; ++e)
            values[e] = (uint32_t)mix64(base ^ (((uint64_t)p << 32) | (uint64_t)(e - offsets[p])));
}

/* x_i = (u32) mix64(mix64(seed) + i) for i in [first, first + n). */
void gen_hash_values(uint64_t seed, uint64_t first, uint64_t n, uint32_t *values)
{
    uint64_t base = mix64(seed);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i)
        values[i] = (uint32_t)mix64(base + first + (uint64_t)i);
}

/* ---- Line-structured text ---- */

/*
 * Text of exactly total_bytes bytes.  Line k has geometric length (success
 * probability 1/(mean+1)) capped at max_len; every line is followed by '\n'.
 * A byte is ' ' with probability space_per_65536 / 65536, else 'a' + v mod 26.
 * The last line is cut so that the final byte is the newline.
 * Pass text == NULL to count lines only.  Returns the number of lines, or
 * (uint64_t)-1 if max_lines is too small.
 */
uint64_t gen_text(uint64_t seed, uint64_t total_bytes, double mean_len, uint32_t max_len,
                  uint32_t space_per_65536, uint8_t *text, uint32_t *starts, uint32_t *lengths,
                  uint64_t max_lines)
{
    uint64_t len_base = mix64(seed ^ 0x11E5ull);
    uint64_t byte_base = mix64(seed ^ 0xB17E5ull);
    double log1mp = log(1.0 - 1.0 / (mean_len + 1.0));
    uint64_t pos = 0, k = 0;
    if (total_bytes == 0) return 0;
    while (pos < total_bytes) {
        uint64_t len = geometric(mix64(len_base + k), log1mp);
        if (len > max_len) len = max_len;
        if (pos + len + 1 > total_bytes) len = total_bytes - 1 - pos;
        if (starts) {
            if (k >= max_lines) return (uint64_t)-1;
            starts[k] = (uint32_t)pos;
            lengths[k] = (uint32_t)len;
        }
        pos += len + 1;
        ++k;
    }
    if (text) {
        #pragma omp parallel for schedule(static)
        for (int64_t w = 0; w < (int64_t)((total_bytes + 3) / 4); ++w) {
            uint64_t r = mix64(byte_base + (uint64_t)w);
            for (int j = 0; j < 4; ++j) {
                uint64_t b = (uint64_t)w * 4 + (uint64_t)j;
                if (b >= total_bytes) break;
                uint32_t v = (uint32_t)(r >> (16 * j)) & 0xFFFFu;
                text[b] = v < space_per_65536 ? (uint8_t)' ' : (uint8_t)('a' + v % 26u);
            }
        }
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)k; ++i)
            text[(uint64_t)starts[i] + lengths[i]] = (uint8_t)'\n';
    }
    return k;
}

/* ---- Graph edges grouped by source vertex ---- */

/*
 * Heavy-tailed out-degrees: d_v = min(cap, floor(beta * (u_v^(-1/alpha) - 1))),
 * u_v uniform in (0, 1], with beta the largest value found by bisection such
 * that sum d_v <= n_edges; the remainder is then handed out one edge at a time
 * to vertices in index order whose degree is in (0, cap).  Writes CSR offsets
 * [n_vertices + 1] and returns beta.
 */
static uint64_t degree_sum(const double *t, uint64_t n, double beta, uint32_t cap)
{
    uint64_t s = 0;
    #pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t v = 0; v < (int64_t)n; ++v) {
        double d = floor(beta * t[v]);
        s += d >= (double)cap ? cap : (uint64_t)d;
    }
    return s;
}

double gen_graph_offsets(uint64_t seed, uint64_t n_vertices, uint64_t n_edges, double alpha,
                         uint32_t cap, double *scratch, uint32_t *offsets)
{
    uint64_t base = mix64(seed);
    #pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < (int64_t)n_vertices; ++v) {
        double u = ((double)(mix64(base + (uint64_t)v) >> 11) + 1.0) * 0x1.0p-53;   /* (0, 1] */
        scratch[v] = pow(u, -1.0 / alpha) - 1.0;
    }
    double lo = 0.0, hi = 1.0;
    while (degree_sum(scratch, n_vertices, hi, cap) <= n_edges && hi < 1e30) hi *= 2.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (degree_sum(scratch, n_vertices, mid, cap) <= n_edges) lo = mid; else hi = mid;
    }
    uint64_t total = 0;
    offsets[0] = 0;
    for (uint64_t v = 0; v < n_vertices; ++v) {
        double d = floor(lo * scratch[v]);
        uint32_t dv = d >= (double)cap ? cap : (uint32_t)d;
        total += dv;
        offsets[v + 1] = dv;   /* degrees for now */
    }
    uint64_t left = n_edges - total;
    int strict = 1;
    while (left > 0) {
        uint64_t before = left;
        for (uint64_t v = 0; v < n_vertices && left > 0; ++v) {
            uint32_t dv = offsets[v + 1];
            if (dv < cap && (dv > 0 || !strict)) { offsets[v + 1] = dv + 1; --left; }
        }
        if (left == before) strict = 0;
        if (left == before && !strict && n_vertices == 0) break;
    }
    for (uint64_t v = 0; v < n_vertices; ++v) offsets[v + 1] += offsets[v];
    return lo;
}

/* Uniform u32 draws from a named sub-stream: out[i] = (u32) mix64(mix64(seed ^ stream) + i). */
void gen_u32_stream(uint64_t seed, uint64_t stream, uint64_t n, uint32_t *out)
{
    uint64_t base = mix64(seed ^ stream);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i)
        out[i] = (uint32_t)mix64(base + (uint64_t)i);
}

/* ---- Batched serving streams ---- */

/*
 * Stream s of a batch: element count n_s = floor(exp(U[ln lo_n, ln hi_n])), mean region
 * length m_s = exp(U[0, ln max_mean]).  Writes n_s and m_s for s in [0, n_streams).
 */
void gen_stream_shapes(uint64_t seed, uint64_t n_streams, double lo_n, double hi_n,
                       double max_mean, uint64_t *n_elems, double *mean_len)
{
    uint64_t base = mix64(seed ^ 0xC5ull);
    for (uint64_t s = 0; s < n_streams; ++s) {
        double u1 = unit_open(mix64(base + 2 * s));
        double u2 = unit_open(mix64(base + 2 * s + 1));
        n_elems[s] = (uint64_t)floor(exp(log(lo_n) + u1 * (log(hi_n) - log(lo_n))));
        mean_len[s] = exp(u2 * log(max_mean));
    }
}

/*
 * Geometric region sizes with the given mean, drawn until they cover n_elems;
 * the last region is cut so the sizes sum to n_elems.  Writes CSR offsets and
 * returns the region count, or (uint64_t)-1 if max_regions is too small.
 * Pass offsets == NULL to count only.
 */
uint64_t gen_geometric_offsets(uint64_t seed, uint64_t n_elems, double mean_len,
                               uint32_t *offsets, uint64_t max_regions)
{
    uint64_t base = mix64(seed ^ 0x5153ull);
    double log1mp = log(1.0 - 1.0 / (mean_len + 1.0));
    uint64_t pos = 0, r = 0;
    if (offsets) offsets[0] = 0;
    while (pos < n_elems) {
        uint64_t len = geometric(mix64(base + r), log1mp);
        if (pos + len > n_elems) len = n_elems - pos;
        pos += len;
        ++r;
        if (offsets) {
            if (r > max_regions) return (uint64_t)-1;
            offsets[r] = (uint32_t)pos;
        }
    }
    return r;
}

/* Poisson arrivals: times[s] = sum of s+1 exponential gaps of the given rate. */
void gen_arrivals(uint64_t seed, uint64_t n, double rate, double *times)
{
    uint64_t base = mix64(seed);
    double t = 0.0;
    for (uint64_t s = 0; s < n; ++s) {
        t += -log(unit_open(mix64(base + s))) / rate;
        times[s] = t;
    }
}
