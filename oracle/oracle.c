/*
 * Serial CPU oracle for region-stateful irregular streaming.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The product path (the
 * HIP library) never calls it and shares no code with it.
 *
 * What it computes is the plain definition of enumeration and aggregation
 * (Timcheck & Buhler, "Streaming Computations with Region-Based State on SIMD
 * Architectures", §4 and §4.1): parents are visited in stream order, each
 * parent's elements are enumerated by index (§4.1, enumeration yields indices
 * and the developer fetches the element under getParent()), every element is
 * passed through the irregular stages in order (§2.1: each input yields zero
 * or more outputs), and the survivors of each region are reduced under that
 * region's context; begin() opens and end() closes every region, so every
 * parent gets exactly one aggregate record, empty parents included (§4.1,
 * the Blob accumulator with begin/run/end).
 *
 * There are no queues, signals, tags or ensembles here.  By Lemma 1 (§3.1)
 * precise signal delivery makes a pipelined run produce exactly this serial
 * result: every item is aggregated under the region that was current when it
 * was emitted.  Queues and ensembles change when work happens, not what is
 * computed; all arithmetic is integer, so the result is unique.
 *
 * The stage kinds are synthetic workloads shaped like the paper's: a sum app
 * over regions of an integer array (§5, cost of regional context), a blob
 * filter feeding an accumulator (§4.1), a line/characters text workload in the
 * manner of the taxi app (§5, comparison of mechanisms) and edges grouped by
 * source vertex (§1 lists this as a region example).
 */
#include <stdint.h>
#include <stddef.h>

#define OR_MODFILTER    1
#define OR_HASH_EXPAND  2
#define OR_TEXT_WORDS   3
#define OR_GRAPH_THRESH 4
#define OR_HASH_TREE    5

#define OR_OK     0
#define OR_EINVAL (-1)
#define OR_ECAP   (-2)

/* MurmurHash3 32-bit finalizer (Appleby, public domain). */
static uint32_t or_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

/* Salted hash used by the hash/expand stages: H(x, s) = fmix32(x ^ (golden * (s + 1))). */
static uint32_t or_hash(uint32_t x, uint32_t salt)
{
    return or_fmix32(x ^ (0x9E3779B9u * (salt + 1u)));
}

uint32_t oracle_fmix32(uint32_t h) { return or_fmix32(h); }
uint32_t oracle_hash(uint32_t x, uint32_t salt) { return or_hash(x, salt); }

/* One region's running aggregate: the state that begin() resets and end() emits. */
typedef struct {
    uint32_t count;
    uint64_t sum;
    uint32_t min;
    uint32_t max;
} or_acc;

static void acc_begin(or_acc *a)
{
    a->count = 0;
    a->sum = 0;
    a->min = 0xFFFFFFFFu;
    a->max = 0;
}

static void acc_run(or_acc *a, uint32_t y)
{
    a->count += 1u;
    a->sum += (uint64_t)y;      /* wraps modulo 2^64 */
    if (y < a->min) a->min = y;
    if (y > a->max) a->max = y;
}

typedef struct {
    or_acc acc;
    uint32_t *out;
    uint64_t out_cap;
    uint64_t n_out;
    int overflow;
} or_sink;

/* The aggregating node receives one surviving item. */
static void sink_item(or_sink *s, uint32_t y)
{
    acc_run(&s->acc, y);
    if (s->out) {
        if (s->n_out < s->out_cap) s->out[s->n_out] = y;
        else s->overflow = 1;
    }
    s->n_out += 1;
}

/*
 * Run one element (enumeration index i of parent p, whose region holds
 * n_p elements starting at 'base') through the stages of 'kind', feeding
 * every surviving item, in order, to the aggregating node.  A tree
 * (OR_HASH_TREE, the tree topologies of §2.1) also feeds a second sink
 * 'second': the filter stage has two children, the expansion (whose
 * outputs reach the first sink) and an aggregating node of its own.
 */
static void run_stages(int kind, const uint32_t *param, const void *elements,
                       uint64_t base, uint32_t n_p, uint32_t i,
                       uint32_t ctx, or_sink *s, or_acc *second)
{
    if (kind == OR_MODFILTER) {
        /* Stage 1 (k = 1): keep x when x mod m equals r. */
        uint32_t x = ((const uint32_t *)elements)[base + i];
        uint32_t m = param[0] ? param[0] : 4u;
        uint32_t r = param[1];
        if (x % m == r) sink_item(s, x);
    } else if (kind == OR_HASH_EXPAND || kind == OR_HASH_TREE) {
        /* Stage 1 (k = 1): keep x when bit 0 of H(x,0) is set. */
        uint32_t x = ((const uint32_t *)elements)[base + i];
        uint32_t h = or_hash(x, 0);
        if (h & 1u) {
            /* The tree's second child of stage 1 aggregates the survivor itself. */
            if (kind == OR_HASH_TREE) acc_run(second, x);
            /* Stage 2 (k = 3): emit c = bits 1..2 of H(x,0) children H(x, j+1), j ascending. */
            uint32_t c = (h >> 1) & 3u;
            for (uint32_t j = 0; j < c; ++j) sink_item(s, or_hash(x, j + 1u));
        }
    } else if (kind == OR_TEXT_WORDS) {
        /* Stage 1 (k = 1): keep index i when byte i starts a word of the line. */
        const uint8_t *b = (const uint8_t *)elements + base;
        if (b[i] != ' ' && (i == 0 || b[i - 1] == ' ')) {
            /* Stage 2 (k = 1): map a word start to the word's length within the line. */
            uint32_t len = 0;
            while (i + len < n_p && b[i + len] != ' ') ++len;
            sink_item(s, len);
        }
    } else if (kind == OR_GRAPH_THRESH) {
        /* Stage 1 (k = 1): keep edge weight w when w < threshold of the source vertex. */
        uint32_t w = ((const uint32_t *)elements)[base + i];
        if (w < ctx) sink_item(s, w);
    }
}

/*
 * oracle_run: the serial definition.
 *
 *   kind          OR_* stage kind
 *   param         4 stage parameters (OR_MODFILTER: modulus, residue)
 *   n_parents     number of parents P
 *   offsets       lengths == NULL: CSR offsets[P+1], region p = [offsets[p], offsets[p+1])
 *                 lengths != NULL: starts[P],     region p = [offsets[p], offsets[p]+lengths[p])
 *   elements      u32 array (kinds 1, 2, 4, 5) or byte array (kind 3) of n_elements entries
 *   parent_param  per-parent context (kind 4: threshold), else NULL
 *   count/sum/min/max   per-parent outputs [P], NULL to skip a field
 *   out, out_cap  optional surviving-item stream in serial order; n_out gets its length
 *
 * Returns OR_OK, OR_EINVAL on a region outside the element array, or OR_ECAP when
 * out_cap is too small (n_out still reports the full length).
 */
static int run_all(int kind, const uint32_t *param, uint64_t n_parents,
                   const uint32_t *offsets, const uint32_t *lengths,
                   const void *elements, uint64_t n_elements,
                   const uint32_t *parent_param,
                   uint32_t *count, uint64_t *sum, uint32_t *min, uint32_t *max,
                   uint32_t *kcount, uint64_t *ksum,
                   uint32_t *out, uint64_t out_cap, uint64_t *n_out)
{
    static const uint32_t zero_param[4] = {0, 0, 0, 0};
    or_sink s;
    or_acc second;
    s.out = out;
    s.out_cap = out_cap;
    s.n_out = 0;
    s.overflow = 0;
    if (!param) param = zero_param;
    if (kind < OR_MODFILTER || kind > OR_HASH_TREE) return OR_EINVAL;
    if (kind == OR_GRAPH_THRESH && !parent_param && n_parents) return OR_EINVAL;

    for (uint64_t p = 0; p < n_parents; ++p) {            /* parents in stream order */
        uint64_t base = offsets[p];
        uint64_t end = lengths ? base + lengths[p] : offsets[p + 1];
        if (end < base || end > n_elements) return OR_EINVAL;
        uint32_t n_p = (uint32_t)(end - base);             /* findCount() */
        uint32_t ctx = parent_param ? parent_param[p] : 0; /* getParent() context */
        acc_begin(&s.acc);                                 /* begin() */
        acc_begin(&second);
        for (uint32_t i = 0; i < n_p; ++i)                 /* enumeration index order */
            run_stages(kind, param, elements, base, n_p, i, ctx, &s, &second);
        if (count) count[p] = s.acc.count;                 /* end(): one record per parent */
        if (sum) sum[p] = s.acc.sum;
        if (min) min[p] = s.acc.min;
        if (max) max[p] = s.acc.max;
        if (kcount) kcount[p] = second.count;              /* the second sink's record */
        if (ksum) ksum[p] = second.sum;
    }
    if (n_out) *n_out = s.n_out;
    return s.overflow ? OR_ECAP : OR_OK;
}

int oracle_run(int kind, const uint32_t *param, uint64_t n_parents,
               const uint32_t *offsets, const uint32_t *lengths,
               const void *elements, uint64_t n_elements,
               const uint32_t *parent_param,
               uint32_t *count, uint64_t *sum, uint32_t *min, uint32_t *max,
               uint32_t *out, uint64_t out_cap, uint64_t *n_out)
{
    return run_all(kind, param, n_parents, offsets, lengths, elements, n_elements, parent_param,
                   count, sum, min, max, NULL, NULL, out, out_cap, n_out);
}

/*
 * oracle_run_tree: as oracle_run, plus the records of the tree's second sink
 * (OR_HASH_TREE): per parent, the count and the sum of the elements that pass
 * the filter stage.
 */
int oracle_run_tree(int kind, const uint32_t *param, uint64_t n_parents,
                    const uint32_t *offsets, const uint32_t *lengths,
                    const void *elements, uint64_t n_elements,
                    const uint32_t *parent_param,
                    uint32_t *count, uint64_t *sum, uint32_t *min, uint32_t *max,
                    uint32_t *kcount, uint64_t *ksum,
                    uint32_t *out, uint64_t out_cap, uint64_t *n_out)
{
    return run_all(kind, param, n_parents, offsets, lengths, elements, n_elements, parent_param,
                   count, sum, min, max, kcount, ksum, out, out_cap, n_out);
}
