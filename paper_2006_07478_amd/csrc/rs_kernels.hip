// gfx950 kernels of the region-stateful streaming pipeline.
//
// One wave64 workgroup is one SIMD processor in the sense of §2.2: it runs a whole
// pipeline instance (enumerating node F, optional second node E, aggregating node A)
// under a non-preemptive scheduler whose state is wave-uniform and lives in scalar
// registers.  It takes parent batches ("claims") from its partition of the launch's
// claims (eight partitions per XCD): most by index, the rest from the partition's
// counter, then from other partitions, returning only when every claim is done.  Under an
// ordered output stream every claim comes from one ascending counter instead (see the
// claim code: the look-back's progress must not depend on which waves are resident).
// A firing consumes an ensemble of at most w = 64*V items: item i sits on lane
// i mod 64 in round i / 64, so one firing is V rounds of 64-lane SIMD work.
//
// Nodes are joined by LDS data queues.  Data-dependent output counts are compacted
// with ballot/mbcnt ranks; every lane writes every round, items that a firing drops
// going to a per-lane spill slot past the queue, so no queue write is predicated.
// Region boundaries travel either
//   - as signals (RS_SIGNAL): each edge has a signal queue S next to its data queue Q
//     (§3.1); an entry is the Q position the signal follows, so the items between two
//     signals are that signal's credit.  A consumer's ensemble never extends past the
//     next signal (the SIMD rule of §3.3) and a node handles a signal only when no item
//     precedes it, running end() for that region.  S is one VGPR, entry n in lane
//     n mod 64, read with readlane and written with a lane select (no LDS round trip); or
//   - as tags (RS_TAG): every queued item carries its region index, ensembles mix
//     regions freely, and the aggregating node reduces by tag (§5); or
//   - as lane-resolved signals (RS_SIGNAL_LANES, the future work of §6): the signals and
//     their queues of RS_SIGNAL, but ensembles may span them, and every node computes each
//     lane's region from the pending signals' positions instead of storing it; or
//   - per stage (RS_ENUM_TAG, the mixed version of §5's taxi comparison): the enumerating
//     node caps every ensemble at its region's end as under signals, and what it emits
//     downstream carries tags.
// The tree kind (RS_HASH_TREE, §2.1's tree topologies) gives the filter node two consumers:
// the expansion and a second aggregating node of its own, whose per-region count and sum
// are kept beside the first sink's records.
//
// An ensemble that is full and inside one region runs its filter and expansion as one
// firing (hash kinds, every strategy): the children go straight into the aggregating
// node's queue and that node takes whole 64-lane rounds, so the scheduler pass and the
// first queue's LDS round trip are paid once per ensemble.  The run of such firings ends
// at the first ensemble that is not full or spans a region end.
//
// Queue depths are launch parameters (a power of two in [2w, 8w]), placed in dynamic LDS
// with the claim's region table and aggregate slots.
// Aggregates are exact integer reductions kept in LDS slots per claim and written once
// per parent; a claim always holds whole regions, so no aggregate is ever shared
// between waves.  How an ensemble reaches the slots depends on the regions it spans: one
// region goes into per-lane accumulators; a few regions of many items each, one wave reduction
// apiece; more regions, per-lane flushes where a lane's items change region, except that under
// tags, when they average 8 or more items, the lanes of a region fold within each 8-lane block
// first, so one lane per block adds to the slot.
//
// Elements reach the enumerating node from HBM through direct buffer->LDS loads into a
// one-ensemble staging slot (16 bytes per lane per load for full ensembles of four or more
// items per lane); the next firing's ensemble is requested as soon as the current one is
// taken, so the loads overlap the downstream firings, and their completion is awaited
// explicitly.  Text is staged the same way, byte windows per firing.  The next claim's
// region table is loaded into registers while the current claim runs, and its first
// ensemble is requested as the current claim ends.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "rs_internal.h"
#include "../../include/regionstream.h"

namespace rs {

// ---------------------------------------------------------------- stage arithmetic

// MurmurHash3's 32-bit finalizer.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

// Salt s of the stage hash: H(x, s) = fmix32(x ^ (0x9E3779B9 * (s + 1))).
__device__ __forceinline__ constexpr uint32_t salt_key(uint32_t s) { return 0x9E3779B9u * (s + 1u); }

// ---------------------------------------------------------------- wave helpers

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Sum of a 64-bit value over the wave's 64 lanes (every lane receives it).
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o, 64);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o, 64);
        v += ((unsigned long long)hi << 32) | lo;
    }
    return v;
}

__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

#define GLOBAL __attribute__((address_space(1)))

// a pointer to device memory, in the global address space
template <class T>
__device__ __forceinline__ GLOBAL T *gbl(T *p) {
    return (GLOBAL T *)p;
}

template <class T>
__device__ __forceinline__ T *uni_ptr(T *p) {
    const uint64_t v = (uint64_t)p;
    return (T *)(((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v));
}

// Lanes of one wave see each other's LDS writes in issue order; this only keeps the
// compiler from moving memory accesses across the point.
__device__ __forceinline__ void order() { asm volatile("" ::: "memory"); }

// LDS byte address of a __shared__ object
__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

// Buffer resource over [base, base + bytes): loads outside the range return zero.
// Base and size are made wave-uniform, so the resource lives in scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(uni_ptr(const_cast<void *>(base)), (short)0, (int)uni(bytes),
                                             0x00020000);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Buffer resource words over [base, base + bytes), wave-uniform: loads outside the range
// return zero.
__device__ __forceinline__ u32x4 rsrc_words(const void *base, uint32_t bytes) {
    const uint64_t b = (uint64_t)uni_ptr(base);
    u32x4 r;
    r.x = (uint32_t)b;
    r.y = (uint32_t)(b >> 32) & 0xFFFFu;
    r.z = uni(bytes);
    r.w = 0x00020000u;
    return r;
}

#define RS_LDSCOPY(off) "buffer_load_dword %[v], %[r], 0 offen offset:" #off " lds\n\t"
#define RS_LDSCOPY4(a, b, c, d) RS_LDSCOPY(a) RS_LDSCOPY(b) RS_LDSCOPY(c) RS_LDSCOPY(d)
#define RS_LDSCOPY16(off) "buffer_load_dwordx4 %[v], %[r], 0 offen offset:" #off " lds\n\t"
#define RS_LDSCOPY_BEGIN "s_nop 2\n\ts_mov_b32 %[s], m0\n\ts_mov_b32 m0, %[m]\n\ts_nop 0\n\t"

// Vector-memory instructions a full ensemble's copy takes (lds_copy below).
template <int V>
constexpr int copy_ops() {
    return V == 1 ? 1 : V == 2 ? 2 : V / 4;
}

// Copies one ensemble's words from the buffer to LDS at lds_base, word i to word i: a full
// ensemble of V >= 4 rounds with one 16-byte load per lane per kilobyte, anything else with one
// 4-byte load per lane per 64 words (the immediate offset advances both addresses).  A partial
// ensemble's range ends inside a 16-byte group, and its 4-byte loads are checked against the
// range one word each.  Written as asm so that the compiler neither orders other LDS accesses
// behind the copy nor waits for it: its completion is awaited explicitly (vmcnt) before the words
// are read; a partial copy takes more instructions than copy_ops<V>(), so a wait sized for a full
// one waits for at least as much.  m0 holds the LDS base and is restored afterwards.  The
// compiler's hazard checks do not look inside asm, so the wait states are part of it: five
// between a vector write of the descriptor's scalar registers (a readfirstlane just before) and
// the loads that read them, and one between the write of m0 and a load into LDS.
template <int V>
__device__ __forceinline__ void lds_copy(u32x4 r, uint32_t lds_base, uint32_t lane, bool full) {
    uint32_t save;
    if constexpr (V >= 4) {
        if (full) {
            if constexpr (V == 4) {
                asm volatile(RS_LDSCOPY_BEGIN RS_LDSCOPY16(0) "s_mov_b32 m0, %[s]"
                             : [s] "=&s"(save) : [v] "v"(lane * 16u), [r] "s"(r), [m] "s"(lds_base) : "memory");
            } else if constexpr (V == 8) {
                asm volatile(RS_LDSCOPY_BEGIN RS_LDSCOPY16(0) RS_LDSCOPY16(1024) "s_mov_b32 m0, %[s]"
                             : [s] "=&s"(save) : [v] "v"(lane * 16u), [r] "s"(r), [m] "s"(lds_base) : "memory");
            } else {
                static_assert(V == 16, "ensemble rounds");
                asm volatile(RS_LDSCOPY_BEGIN RS_LDSCOPY16(0) RS_LDSCOPY16(1024) RS_LDSCOPY16(2048)
                             RS_LDSCOPY16(3072) "s_mov_b32 m0, %[s]"
                             : [s] "=&s"(save) : [v] "v"(lane * 16u), [r] "s"(r), [m] "s"(lds_base) : "memory");
            }
            return;
        }
    }
    if constexpr (V == 1) {
        asm volatile(RS_LDSCOPY_BEGIN RS_LDSCOPY(0) "s_mov_b32 m0, %[s]"
                     : [s] "=&s"(save) : [v] "v"(lane * 4u), [r] "s"(r), [m] "s"(lds_base) : "memory");
    } else if constexpr (V == 2) {
        asm volatile(RS_LDSCOPY_BEGIN RS_LDSCOPY(0) RS_LDSCOPY(256) "s_mov_b32 m0, %[s]"
                     : [s] "=&s"(save) : [v] "v"(lane * 4u), [r] "s"(r), [m] "s"(lds_base) : "memory");
    } else if constexpr (V == 4) {
        asm volatile(RS_LDSCOPY_BEGIN RS_LDSCOPY4(0, 256, 512, 768)
                     "s_mov_b32 m0, %[s]"
                     : [s] "=&s"(save) : [v] "v"(lane * 4u), [r] "s"(r), [m] "s"(lds_base) : "memory");
    } else if constexpr (V == 8) {
        asm volatile(RS_LDSCOPY_BEGIN RS_LDSCOPY4(0, 256, 512, 768)
                     RS_LDSCOPY4(1024, 1280, 1536, 1792) "s_mov_b32 m0, %[s]"
                     : [s] "=&s"(save) : [v] "v"(lane * 4u), [r] "s"(r), [m] "s"(lds_base) : "memory");
    } else {
        asm volatile(RS_LDSCOPY_BEGIN RS_LDSCOPY4(0, 256, 512, 768)
                     RS_LDSCOPY4(1024, 1280, 1536, 1792) RS_LDSCOPY4(2048, 2304, 2560, 2816)
                     RS_LDSCOPY4(3072, 3328, 3584, 3840) "s_mov_b32 m0, %[s]"
                     : [s] "=&s"(save) : [v] "v"(lane * 4u), [r] "s"(r), [m] "s"(lds_base) : "memory");
    }
}

// Slot of queue position base + i in a ring of d slots, where base < d and i < d: one
// conditional subtraction, written as an unsigned minimum.
__device__ __forceinline__ uint32_t qslot(uint32_t d, uint32_t base, uint32_t i) {
    const uint32_t p = base + i;
    return min(p, p - d);
}

// a where the lane's bit of mask is set, else b (one v_cndmask, never a branch).  The mask is
// first copied to a scalar register pair of the asm's own: the compiler may otherwise hand
// over exec itself (a ballot of a condition true on every lane folds to it), and a v_cndmask
// that takes exec as its lane mask selects wrongly on the upper half of the wave.  The copy
// also keeps the select clear of the wait states that a vector write of the mask (a compare)
// would need before a vector read, which the compiler cannot see inside asm.
__device__ __forceinline__ uint32_t pick(uint64_t mask, uint32_t a, uint32_t b) {
    uint32_t r;
    uint64_t m;
    asm("s_mov_b64 %1, %4\n\tv_cndmask_b32 %0, %2, %3, %1" : "=v"(r), "=&s"(m) : "v"(b), "v"(a), "s"(mask));
    return r;
}

// Wait until at most N vector-memory operations of this wave are outstanding; also a
// compiler barrier, so no memory access moves across it.
template <int N>
__device__ __forceinline__ void wait_vmem() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Bit 7 of each byte of the result is set where that byte of w is a space (0x20), exactly: the
// sum inside never carries from one byte into the next.
__device__ __forceinline__ uint32_t space_bytes(uint32_t w) {
    const uint32_t z = w ^ 0x20202020u;
    return ~(((z & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | z) & 0x80808080u;
}

template <bool B>
struct BoolC {
    static constexpr bool value = B;
};

// Exclusive prefix of per-item counts n[k] (0..3) over an ensemble laid out as item
// k*64 + lane, in that order.  off[k] is the item's first output slot relative to the
// firing's base; the return value is the firing's output count (uniform).
template <int V, bool TWO_BITS>
__device__ __forceinline__ uint32_t ens_scan(const uint32_t (&n)[V], uint32_t (&off)[V]) {
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const uint64_t b0 = __ballot(n[k] & 1u);
        uint32_t within = rank_below(b0);
        uint32_t wsum = (uint32_t)__popcll(b0);
        if constexpr (TWO_BITS) {
            const uint64_t b1 = __ballot((n[k] >> 1) & 1u);
            within += 2u * rank_below(b1);
            wsum += 2u * (uint32_t)__popcll(b1);
        }
        off[k] = run + within;
        run += wsum;
    }
    return uni(run);
}

struct Acc {
    uint32_t cnt;
    unsigned long long sum;
    uint32_t mn, mx;
};

__device__ __forceinline__ void acc_reset(Acc &a) {
    a.cnt = 0;
    a.sum = 0;
    a.mn = 0xFFFFFFFFu;
    a.mx = 0;
}
// Adds y when act holds, without a branch.
__device__ __forceinline__ void acc_add(Acc &a, uint32_t y, bool act) {
    a.cnt += act ? 1u : 0u;
    a.sum += (unsigned long long)(act ? y : 0u);
    const uint32_t lo = act ? y : 0xFFFFFFFFu, hi = act ? y : 0u;
    a.mn = a.mn < lo ? a.mn : lo;
    a.mx = a.mx > hi ? a.mx : hi;
}

// x moved across lanes by one DPP control; lanes with no source in the pattern (or in rows
// outside row_mask) get id instead.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_or(uint32_t id, uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)x, CTRL, ROW_MASK, 0xF, false);
}

// One step of the lane-63 reduction for all four fields.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void acc_dpp_step(Acc &a) {
    const uint32_t c = dpp_or<CTRL, ROW_MASK>(0u, a.cnt);
    const uint32_t lo = dpp_or<CTRL, ROW_MASK>(0u, (uint32_t)a.sum);
    const uint32_t hi = dpp_or<CTRL, ROW_MASK>(0u, (uint32_t)(a.sum >> 32));
    const uint32_t mn = dpp_or<CTRL, ROW_MASK>(0xFFFFFFFFu, a.mn);
    const uint32_t mx = dpp_or<CTRL, ROW_MASK>(0u, a.mx);
    a.cnt += c;
    a.sum += ((unsigned long long)hi << 32) | lo;
    a.mn = a.mn < mn ? a.mn : mn;
    a.mx = a.mx > mx ? a.mx : mx;
}

// Wave reduction of per-lane accumulators into wave-uniform values, with DPP moves only (no LDS
// crossbar): an inclusive scan within each row of 16 lanes (shifts by 1, 2, 4, 8), then the
// row totals carried across rows by the row broadcasts of lane 15 and lane 31; lane 63 ends
// with the total, which is read into scalar registers.  Must run with every lane active.
__device__ __forceinline__ Acc wave_reduce(Acc a) {
    acc_dpp_step<0x111, 0xF>(a);   // row_shr:1
    acc_dpp_step<0x112, 0xF>(a);   // row_shr:2
    acc_dpp_step<0x114, 0xF>(a);   // row_shr:4
    acc_dpp_step<0x118, 0xF>(a);   // row_shr:8
    acc_dpp_step<0x142, 0xA>(a);   // row_bcast:15 into rows 1 and 3
    acc_dpp_step<0x143, 0xC>(a);   // row_bcast:31 into rows 2 and 3
    Acc r;
    // readlane yields an int: each half goes through uint32_t so the low half is not
    // sign-extended into the high one
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((uint32_t)a.sum, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((uint32_t)(a.sum >> 32), 63);
    r.cnt = (uint32_t)__builtin_amdgcn_readlane(a.cnt, 63);
    r.sum = ((unsigned long long)hi << 32) | lo;
    r.mn = (uint32_t)__builtin_amdgcn_readlane(a.mn, 63);
    r.mx = (uint32_t)__builtin_amdgcn_readlane(a.mx, 63);
    return r;
}

// Segmented inclusive scans inside 8-lane blocks, one field at a time: t1/t2/t4 say whether
// lane t takes in lane t - 1/2/4's partial (that lane is in its block and carries the same key;
// keys grow along the lanes, so an equal key some lanes back means the same segment).  Identity
// values fill the lanes a shift reaches outside its row.
template <int OP>   // 0: add, 1: min, 2: max
__device__ __forceinline__ uint32_t seg_scan32(uint32_t v, bool t1, bool t2, bool t4) {
    constexpr uint32_t ID = OP == 1 ? 0xFFFFFFFFu : 0u;
    auto comb = [](uint32_t a, uint32_t b) { return OP == 0 ? a + b : OP == 1 ? min(a, b) : max(a, b); };
    uint32_t p = dpp_or<0x111, 0xF>(ID, v);   // row_shr:1
    v = t1 ? comb(v, p) : v;
    p = dpp_or<0x112, 0xF>(ID, v);            // row_shr:2
    v = t2 ? comb(v, p) : v;
    p = dpp_or<0x114, 0xF>(ID, v);            // row_shr:4
    return t4 ? comb(v, p) : v;
}
// The 64-bit sum as two 16-bit halves, each summed in 32 bits (a block has at most 8 lanes)
__device__ __forceinline__ unsigned long long seg_sum64(uint32_t v, bool t1, bool t2, bool t4) {
    const uint32_t lo = seg_scan32<0>(v & 0xFFFFu, t1, t2, t4), hi = seg_scan32<0>(v >> 16, t1, t2, t4);
    return ((unsigned long long)hi << 16) + lo;
}

// Set bits among ensemble indices [0, rel) of the per-round masks m (index k*64 + lane is bit
// lane of m[k]); rel is per lane, at most 64*V.
template <int V>
__device__ __forceinline__ uint32_t bits_below(const uint64_t (&m)[V], uint32_t rel) {
    uint32_t n = 0;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const uint32_t lo = (uint32_t)k * 64u;
        const uint32_t r = rel > lo ? min(rel - lo, 64u) : 0u;
        const uint64_t low = r >= 64u ? ~0ull : ((1ull << r) - 1ull);
        n += (uint32_t)__popcll(m[k] & low);
    }
    return n;
}

// ---------------------------------------------------------------- geometry

template <int V>
struct Geo {
    static constexpr uint32_t EW = 64u * V;   // ensemble width: items one firing consumes
    static constexpr uint32_t SQ = 64u;       // signal queue capacity (the finite S of §3.1)
    static constexpr uint32_t R = 4u;         // region-table rows per lane (256 entries)
};

// Data-queue depths for queue depth q (the pipeline's queue_depth: a power of two, at least 2w):
// the queue in front of the second node holds q items; the one in front of the third node holds
// q, and one ensemble more behind the expansion (its consumer drains it below one ensemble
// before the expansion fires, so room for one full ensemble's worst case of 3w on top lets the
// expansion always fire full ensembles; at q = 2w that is the 3w of that argument).
// The hash stages, linear (RS_HASH_EXPAND) or in the tree whose filter also feeds a second sink
// (RS_HASH_TREE).
__host__ __device__ inline bool hash_kind(uint32_t kind) { return kind == RS_HASH_EXPAND || kind == RS_HASH_TREE; }

__host__ __device__ inline uint32_t depth2(uint32_t kind, uint32_t ew, uint32_t q) {
    return hash_kind(kind) ? q + ew : kind == RS_TEXT_WORDS ? q : 1u;
}

// LDS arrays sized at launch: the data queues (for the queue depth q), each followed by 64
// spill slots (one per lane) for dropped items, and the per-claim arrays for the batch's largest
// claim (bmax parents).  Fused firings (hash kind) use the third node's queue as a plain array of
// 3w + 66 slots (a leftover of under 64 items, up to 3w children and two slots a firing may write
// past its last child) followed by 66 dump slots.
struct Dyn {
    uint32_t q1v, q2v, q1a, q1t, q2t, sum, ksum, vt, sx, cx, cnt, mn, mx, kcnt, bytes;
};
__host__ __device__ inline Dyn dyn_layout(uint32_t kind, uint32_t strategy, uint32_t ew, uint32_t q, uint32_t bmax) {
    const bool tag = strategy == RS_TAG || strategy == RS_ENUM_TAG;   // items carry tags
    const bool has_e = hash_kind(kind) || kind == RS_TEXT_WORDS;
    const uint32_t d2 = depth2(kind, ew, q);
    uint32_t q2 = has_e ? d2 + 64u : 0u;
    if (hash_kind(kind) && q2 < 3u * ew + 132u) q2 = 3u * ew + 132u;
    Dyn d;
    uint32_t o = 0;
    d.sum = o;
    o += 8u * bmax;   // u64 slots first (8-byte aligned)
    d.ksum = o;       // the tree's second sink
    if (kind == RS_HASH_TREE) o += 8u * bmax;
    d.q1v = o;
    o += 4u * (q + 64u);
    d.q2v = o;
    o += 4u * q2;
    d.vt = o;
    o += 4u * (bmax + 1u);
    d.sx = o;
    if (kind == RS_TEXT_WORDS) o += 4u * bmax;
    d.cx = o;
    if (kind == RS_GRAPH_THRESH) o += 4u * bmax;
    d.cnt = o;
    o += 4u * bmax;
    d.mn = o;
    o += 4u * bmax;
    d.mx = o;
    o += 4u * bmax;
    d.kcnt = o;
    if (kind == RS_HASH_TREE) o += 4u * bmax;
    d.q1a = o;
    if (hash_kind(kind)) o += q + 64u;
    d.q1t = o;
    if (tag) o += q + 64u;
    d.q2t = o;
    if (tag && has_e) o += d2 + 64u;
    d.bytes = (o + 15u) & ~15u;
    return d;
}

// A stream-table entry held in scalar registers: every field is read once and made
// wave-uniform, so buffer resources and loop bounds built from it need no per-lane handling.
// Its pointers are in the global address space, so accesses through them are global (not flat)
// instructions: flat accesses also count against the LDS wait counter, and would make every
// later LDS wait wait for them.
struct SDesc {
    const uint8_t *elements;
    const GLOBAL uint32_t *offsets, *lengths, *pparam;
    GLOBAL uint32_t *agg_count, *agg_min, *agg_max, *agg_kcount, *out_items;
    GLOBAL unsigned long long *agg_sum, *agg_ksum, *lookback, *stats;
    uint32_t n_parents, n_elements, B, claim_begin;
};
__device__ __forceinline__ SDesc load_sdesc(const StreamDev &s) {
    SDesc d;
    d.elements = uni_ptr((const uint8_t *)s.elements);
    d.offsets = gbl(uni_ptr(s.offsets));
    d.lengths = gbl(uni_ptr(s.lengths));
    d.pparam = gbl(uni_ptr(s.pparam));
    d.agg_count = gbl(uni_ptr(s.agg_count));
    d.agg_sum = gbl(uni_ptr(s.agg_sum));
    d.agg_min = gbl(uni_ptr(s.agg_min));
    d.agg_max = gbl(uni_ptr(s.agg_max));
    d.agg_kcount = gbl(uni_ptr(s.agg_kcount));
    d.agg_ksum = gbl(uni_ptr(s.agg_ksum));
    d.out_items = gbl(uni_ptr(s.out_items));
    d.lookback = gbl(uni_ptr(s.lookback));
    d.stats = gbl(uni_ptr(s.stats));
    d.n_parents = uni(s.n_parents);
    d.n_elements = uni(s.n_elements);
    d.B = uni(s.parents_per_claim);
    d.claim_begin = uni(s.claim_begin);
    return d;
}

// Region table of one claim, as loaded from HBM: lane t holds parents p0 + r*64 + t.
template <int R>
struct ClaimRegs {
    uint32_t off[R];   // CSR offsets[p0 + i] (i <= nb), or start of region p0 + i (i < nb)
    uint32_t len[R];   // length of region p0 + i (start+length streams)
    uint32_t ctx[R];   // per-parent context
    uint32_t nb;                 // parents in the claim (uniform)
    const uint8_t *elements;     // its stream's element array (uniform)
    uint32_t n_elements;         // and that array's size
};

// ---------------------------------------------------------------- the pipeline kernel

template <int KIND, int STRAT, int V>
__global__ void __launch_bounds__(64) rs_pipeline(LaunchArgs a) {
    constexpr bool TAG = (STRAT == RS_TAG);
    // lane-resolved signals: ensembles span region boundaries, the boundaries travel on the
    // signal queues only, and every node computes each lane's region from the pending signals
    constexpr bool LANES = (STRAT == RS_SIGNAL_LANES);
    // per-stage choice (the second taxi version of §5): the enumerating node walks one region at a
    // time, as under signals, and tags each item it emits with that region; downstream nodes work
    // as under tags, their ensembles spanning regions
    constexpr bool HYB = (STRAT == RS_ENUM_TAG);
    // the enumerating node walks consecutive positions (tags, lane-resolved signals); under
    // signals and the per-stage choice it walks one region at a time
    constexpr bool WALK = TAG || LANES;
    constexpr bool TAGQ = TAG || HYB;                    // queued items carry their region's tag
    constexpr bool SIGQ = (STRAT == RS_SIGNAL);          // signals cap every downstream ensemble
    constexpr bool PERLANE = WALK || HYB;                // the aggregating node resolves regions per lane
    constexpr bool HASHK = (KIND == RS_HASH_EXPAND || KIND == RS_HASH_TREE);
    // the tree topology: the filter (the enumerating node) has two children, the expansion and an
    // aggregating node of its own, which sums the filter's survivors per region
    constexpr bool TREE = (KIND == RS_HASH_TREE);
    constexpr bool HAS_E = (HASHK || KIND == RS_TEXT_WORDS);
    constexpr bool BYTES = (KIND == RS_TEXT_WORDS);
    constexpr bool CTXP = (KIND == RS_GRAPH_THRESH);
    constexpr uint32_t KE = HASHK ? 3u : 1u;   // outputs per input of E, at most
    using G = Geo<V>;
    constexpr uint32_t EW = G::EW, SQ = G::SQ, R = G::R;
    const uint32_t D1 = a.qdepth;                       // data slots in front of the second node
    const uint32_t D2 = depth2(KIND, EW, D1);           // in front of the third node
    const uint32_t DA = HAS_E ? D2 : D1;                // the aggregating node's input queue
    static_assert(!LANES || (KIND != RS_TEXT_WORDS && V <= 4), "lane-resolved signals: u32 kinds, w <= 256");
    constexpr bool FUSE = HASHK;   // fused firings, below
    constexpr uint32_t FL = 3u * EW + 66u, FDUMP = FL;

    // text: a firing's bytes from the word before its first address, in 1, 1, 2, 4 or 8 copies of
    // 256 bytes (at least w + 8 bytes)
    constexpr uint32_t TB = V <= 2 ? 256u : 2u * EW;
    // text under tags: two windows of TWB bytes, alternating (a window holds TWB / w firings: four,
    // or sixteen at w = 64; measured best among 1, 2 and 4 KB at w = 256 and 512)
    constexpr uint32_t TWB = EW < 256u ? 1024u : 4u * EW;
    __shared__ uint32_t fsl[BYTES ? (TAG ? 2u * TWB / 4u : TB / 4u) : EW];   // staging for the enumerating node
    extern __shared__ __attribute__((aligned(16))) uint8_t dyn[];

    const Dyn lay = dyn_layout(KIND, STRAT, EW, D1, a.bmax);
    uint32_t *const q1v = (uint32_t *)(dyn + lay.q1v);
    uint8_t *const q1a = dyn + lay.q1a;                 // the expansion's child count per item
    uint8_t *const q1t = dyn + lay.q1t;                 // tags
    uint32_t *const q2v = (uint32_t *)(dyn + lay.q2v);
    uint8_t *const q2t = dyn + lay.q2t;
    unsigned long long *const s_sum = (unsigned long long *)(dyn + lay.sum);
    uint32_t *const VT = (uint32_t *)(dyn + lay.vt);    // region starts in enumeration order, end at [nb]
    uint32_t *const SX = (uint32_t *)(dyn + lay.sx);    // region start addresses (start+length streams)
    uint32_t *const CX = (uint32_t *)(dyn + lay.cx);    // per-parent context
    uint32_t *const s_cnt = (uint32_t *)(dyn + lay.cnt);
    uint32_t *const s_min = (uint32_t *)(dyn + lay.mn);
    uint32_t *const s_max = (uint32_t *)(dyn + lay.mx);
    uint32_t *const s_kcnt = (uint32_t *)(dyn + lay.kcnt);                       // tree: second sink
    unsigned long long *const s_ksum = (unsigned long long *)(dyn + lay.ksum);

    const uint32_t t = threadIdx.x;
    GLOBAL uint32_t *const ctl = gbl(a.ctl);

    // stage parameters
    const uint32_t modm = a.param[0] ? a.param[0] : 4u;
    const uint32_t modr = a.param[1];
    const bool mod_pow2 = (modm & (modm - 1u)) == 0u;

    // this launch's epoch (set by the reset kernel before it), as a 24-bit tag in
    // [1, 2^24 - 1] for the look-back words
    const uint32_t epoch_tag =
        uni(__hip_atomic_load(&ctl[CTL_EPOCH], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) % 0xFFFFFFu + 1u;

    // stream of global claim gg: the last with claim_begin <= gg
    auto stream_of = [&](uint32_t gg) -> uint32_t {
        uint32_t lo = 0, hi = a.n_streams;
        while (hi - lo > 1u) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.streams[mid].claim_begin <= gg) lo = mid; else hi = mid;
        }
        return uni(lo);
    };
    // the stream-table entry last used, copied to LDS (consecutive claims usually share a
    // stream); fields are read from it where they are needed, which keeps scalar registers free
    __shared__ StreamDev sdl;
    uint32_t sdl_idx = 0xFFFFFFFFu;
    auto ensure_sd = [&](uint32_t si) {
        if (si != sdl_idx) {
            constexpr uint32_t NW = sizeof(StreamDev) / 4u;
            static_assert(sizeof(StreamDev) % 4u == 0u && NW <= 64u, "one word per lane");
            uint32_t v = 0;
            if (t < NW) v = gbl((const uint32_t *)&a.streams[si])[t];
            if (t < NW) ((uint32_t *)&sdl)[t] = v;
            order();
            sdl_idx = si;
        }
    };
    // this lane's share of the region table of claim gg (loads only; consumed a claim later)
    // r.nb, r.elements and r.n_elements: the claim's parent count and its stream's element array
    auto load_claim = [&](uint32_t gg, ClaimRegs<R> &r) {
#pragma unroll
        for (uint32_t q = 0; q < R; ++q) r.off[q] = r.len[q] = r.ctx[q] = 0;
        r.nb = 0;
        r.elements = nullptr;
        r.n_elements = 0;
        if (gg >= a.total_claims) return;
        ensure_sd(stream_of(gg));
        const SDesc sd = load_sdesc(sdl);
        const uint32_t B = sd.B;
        const uint32_t p0 = (gg - sd.claim_begin) * B;
        const uint32_t nb = min(B, sd.n_parents - p0);
        r.nb = nb;
        r.elements = sd.elements;
        r.n_elements = sd.n_elements;
#pragma unroll
        for (uint32_t q = 0; q < R; ++q) {
            const uint32_t i = q * 64u + t;
            if constexpr (!BYTES) {
                if (i <= nb) r.off[q] = sd.offsets[p0 + i];
            } else {
                if (i < nb) {
                    r.off[q] = sd.offsets[p0 + i];
                    r.len[q] = sd.lengths[p0 + i];
                }
            }
            if constexpr (CTXP) {
                if (i < nb) r.ctx[q] = sd.pparam[p0 + i];
            }
        }
    };
    // Claims.  The launch's claims are split into n_parts contiguous partitions, each served by
    // the waves of one XCD (workgroups are dispatched round-robin over the 8 XCDs, and wave b's
    // partition is b mod 64), each with its own counter in its own cache line, so claim traffic
    // spreads over independent atomics and no counter sees more than a few dozen waves.  A wave first takes
    // about seven eighths of its home partition's claims by its index (claims widx,
    // widx + Wp, widx + 2 Wp, ... for the partition's Wp waves; no atomic at all), then claims
    // from its home counter, and when that partition is used up, from the other partitions'
    // counters, found with one read of all of them.
    //
    // An ordered output stream is different: a claim waits in its look-back on every claim before
    // it, so a claim must never belong to a wave that has not started.  Its claims come from one
    // ascending counter only (one partition, none by index), so the claims taken at any moment are
    // a prefix of the claim order and each belongs to a running wave; the smallest unfinished
    // claim is then the current claim of a running wave, and every claim before it has published
    // its count, whatever number of the launch's waves are resident.
    const uint32_t n_claims = a.total_claims, np = a.n_parts, n_waves = gridDim.x;
    const bool by_index = a.emit_outputs == 0u;
    const uint32_t np_log = np == 1u ? 0u : 6u;   // n_parts is 1 or CTL_NPART = 64
    const uint32_t home = blockIdx.x & (np - 1u), widx = blockIdx.x >> np_log;
    auto p_begin = [&](uint32_t q) -> uint32_t { return (uint32_t)(((uint64_t)n_claims * q) >> np_log); };
    auto p_waves = [&](uint32_t q) -> uint32_t { return n_waves > q ? ((n_waves - 1u - q) >> np_log) + 1u : 0u; };
    // claims each wave of partition q takes by index (at least two: the two claims in hand)
    auto p_static = [&](uint32_t q) -> uint32_t {
        const uint32_t wq = p_waves(q), size = p_begin(q + 1u) - p_begin(q);
        return (wq && by_index) ? max(2u, size / 8u * 7u / wq) : 0u;
    };
    const uint32_t home_static = p_static(home), home_waves = p_waves(home);
    const uint32_t home_begin = p_begin(home), home_end = p_begin(home + 1u);
    uint32_t n_static = 0;
    uint64_t dry = 0;   // partitions found without dynamic claims left
    auto take_claim = [&]() -> uint32_t {
        while (n_static < home_static) {
            const uint32_t c = home_begin + widx + n_static * home_waves;
            ++n_static;
            if (c < home_end) return c;
            n_static = home_static;
        }
        // dynamic claims: the home counter until it runs dry, then one read of every
        // partition's counter (lane q reads partition q) finds the partitions with claims left
        while (true) {
            uint32_t q = home;
            if ((dry & (1ull << home)) != 0ull) {
                uint32_t left = 0;
                if (t < np) {
                    const uint32_t f = p_begin(t) + p_static(t) * p_waves(t), e2 = p_begin(t + 1u);
                    left = f < e2 && __hip_atomic_load(&ctl[CTL_PART + t * CTL_PART_STRIDE], __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT) < e2 - f;
                }
                const uint64_t m = __ballot(left) & ~dry;
                if (!m) return n_claims;   // nothing left
                q = (uint32_t)__builtin_ctzll(m);
            }
            const uint32_t first = p_begin(q) + p_static(q) * p_waves(q), end = p_begin(q + 1u);
            uint32_t got = 0xFFFFFFFFu;
            if (first < end && t == 0) {
                const uint32_t k = __hip_atomic_fetch_add(&ctl[CTL_PART + q * CTL_PART_STRIDE], 1u, __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT);
                if (k < end - first) got = first + k;
            }
            got = uni(got);
            if (got != 0xFFFFFFFFu) return got;
            dry |= 1ull << q;
        }
    };

    // claims are taken two ahead: g is worked on, g1 is next (its region table in registers).
    // Under an ordered output stream this keeps the look-back's progress: the wave holding a
    // claim is running, and it works its claims in increasing order.
    uint32_t g = take_claim();
    uint32_t g1 = take_claim();
    ClaimRegs<R> cur;
    load_claim(g, cur);
    // claim whose first ensemble the staging slot receives, requested as the previous claim ended
    // (u32 kinds), so that a claim does not start with a full memory round trip
    uint32_t pf_g = 0xFFFFFFFFu;

    while (g < a.total_claims) {
        const uint32_t g_next = take_claim();   // the claim after g1
        ClaimRegs<R> nxt;
        load_claim(g1, nxt);                    // consumed at the next claim

        ensure_sd(stream_of(g));
        const SDesc sd = load_sdesc(sdl);
        const uint8_t *const elems = sd.elements;
        const uint32_t B = sd.B;
        const uint32_t cidx = g - sd.claim_begin;
        const uint32_t p0 = cidx * B;
        const uint32_t nb = uni(min(B, sd.n_parents - p0));

        // ---- region table of the claim (enumeration: findCount per parent)
        uint32_t vbeg, vend;
        if constexpr (!BYTES) {
#pragma unroll
            for (uint32_t q = 0; q < R; ++q) {
                const uint32_t i = q * 64u + t;
                if (i <= nb) VT[i] = cur.off[q];
                if constexpr (CTXP)
                    if (i < nb) CX[i] = cur.ctx[q];
            }
            order();
            vbeg = uni(VT[0]);
            vend = uni(VT[nb]);
        } else {
            // enumeration positions of the lines: exclusive prefix of their lengths
            uint32_t carry = 0;
#pragma unroll
            for (uint32_t q = 0; q < R; ++q) {
                const uint32_t i = q * 64u + t;
                const uint32_t len = i < nb ? cur.len[q] : 0u;
                uint32_t inc = len;
#pragma unroll
                for (uint32_t o = 1; o < 64; o <<= 1) {
                    const uint32_t u = __shfl_up(inc, o, 64);
                    if (t >= o) inc += u;
                }
                if (i < nb) {
                    SX[i] = cur.off[q];
                    VT[i] = carry + inc - len;
                }
                carry += uni(__shfl(inc, 63, 64));
            }
            if (t == 0) VT[nb] = carry;
            order();
            vbeg = 0;
            vend = carry;
            if constexpr (WALK) {   // lines are enumerated over the claim's byte address range
                vbeg = nb ? uni(SX[0]) : 0u;
                vend = nb ? uni(SX[nb - 1] + (VT[nb] - VT[nb - 1])) : 0u;
            }
        }
        for (uint32_t i = t; i < nb; i += 64u) {
            s_cnt[i] = 0;
            s_sum[i] = 0ull;
            s_min[i] = 0xFFFFFFFFu;
            s_max[i] = 0;
            if constexpr (TREE) {
                s_kcnt[i] = 0;
                s_ksum[i] = 0ull;
            }
        }

        // The claim's regions must be ordered and inside the element array before any element
        // is read; a malformed stream is flagged and its claims are skipped.
        {
            bool bad = false;
            for (uint32_t i = t; i < nb; i += 64u) {
                if constexpr (!BYTES) {
                    bad |= (VT[i] > VT[i + 1]) || (i + 1u == nb && VT[nb] > sd.n_elements);
                } else {
                    const unsigned long long end = (unsigned long long)SX[i] + (VT[i + 1] - VT[i]);
                    const unsigned long long lim = (i + 1u < nb) ? SX[i + 1] : sd.n_elements;
                    bad |= end > lim;
                }
            }
            if (__ballot(bad)) {
                if (t == 0) {
                    __hip_atomic_fetch_or((GLOBAL unsigned int *)&sd.stats[ST_ERROR], 1u, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_fetch_or(&ctl[CTL_BAD], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (a.emit_outputs)   // successors of this claim must not wait for it
                        __hip_atomic_store(&sd.lookback[cidx], ((unsigned long long)epoch_tag << 40) | (2ull << 38),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                order();
                g = g1;
                g1 = g_next;
                cur = nxt;
                continue;
            }
        }

        // ---- element access
        // text: the whole byte array (addresses fit in 32 bits); word loads near its end fall
        // back to bytes, so no load depends on the range check for its value
        const __amdgpu_buffer_rsrc_t rtext = rsrc(elems, BYTES ? sd.n_elements : 0u);
        // u32 elements: the ensemble starting at position pos is copied to the staging slot by
        // direct buffer->LDS loads (item k*64 + lane to word k*64 + lane; positions past vend
        // read as zero).  A firing requests the next firing's ensemble as soon as it has taken
        // the slot's contents into registers, so the copy overlaps whatever fires in between;
        // its completion is awaited explicitly (vmcnt) before the slot is read.  One slot, not
        // two: the LDS it saves buys more resident waves, which hide the latency better.
        uint32_t spos = pf_g == g ? vbeg : 0xFFFFFFFFu;   // position whose ensemble the slot holds or receives
        auto stage = [&](uint32_t pos) {
            if constexpr (!BYTES) {
                spos = 0xFFFFFFFFu;
                if (pos < vend) {
                    lds_copy<V>(rsrc_words(elems + (size_t)pos * 4u, min(EW, vend - pos) * 4u), uni(lds_addr(fsl)),
                                t, vend - pos >= EW);
                    spos = pos;
                }
            }
        };
        // text: the window of bytes [tsbase, tsbase + TB) holding the firing at address tspos, from
        // the word before it (for the byte before the first); bytes past the array read as zero
        uint32_t tspos = 0xFFFFFFFFu, tsbase = 0;
        auto stage_text = [&](uint32_t adr) {
            if constexpr (BYTES) {
                const uint32_t base = adr >= 4u ? (adr & ~3u) - 4u : 0u;
                tspos = adr;
                tsbase = base;
                if (base < sd.n_elements)
                    lds_copy<TB / 256u>(rsrc_words(elems + base, min(TB, sd.n_elements - base)), uni(lds_addr(fsl)), t,
                                        false);
            }
        };
        // Text under tags: the claim's bytes from tr_f0 on, in windows of TWB bytes (window m in
        // buffer m mod 2).  A firing never straddles two windows (w divides TWB and firings start
        // at tr_f0 + k w); the first firing of window m waits for it, keeps the last word of window
        // m - 1 (the byte before its first), and requests window m + 1 into the buffer m - 1 held,
        // so a window's copy overlaps the TWB / w firings of the window before it.
        uint32_t tr_f0 = 0, tr_m = 0xFFFFFFFFu, tr_carry = 0x20202020u;
        auto tring_request = [&](uint32_t m) {
            if constexpr (BYTES && TAG) {
                const uint32_t wb = tr_f0 + m * TWB;
                if (wb < vend) {
                    const uint32_t nbytes = min(TWB, sd.n_elements - wb);
                    lds_copy<TWB / 256u>(rsrc_words(elems + wb, nbytes), uni(lds_addr(fsl + (m & 1u) * (TWB / 4u))), t,
                                         nbytes == TWB);
                }
            }
        };
        // u32 elements outside the staged path (the output-count pass): plain buffer loads
        auto load_ens = [&](uint32_t pos, uint32_t n, uint32_t (&x)[V]) {
            const __amdgpu_buffer_rsrc_t r = rsrc(elems + (size_t)pos * 4u, n * 4u);
#pragma unroll
            for (int k = 0; k < V; ++k) x[k] = __builtin_amdgcn_raw_buffer_load_b32(r, (k * 64 + t) * 4, 0, 0);
        };

        // Region of enumeration position v (tag strategy): the largest j whose start is <= v,
        // by element index (CSR) or by byte address (lines), searching from jlo_.
        auto f_region = [&](uint32_t v, uint32_t jlo_) -> uint32_t {
            const uint32_t *key = BYTES ? SX : VT;
            uint32_t l2 = jlo_, h2s = nb;
            while (h2s - l2 > 1u) {
                const uint32_t m = (l2 + h2s) >> 1;
                if (key[m] <= v) l2 = m; else h2s = m;
            }
            return l2;
        };
        // Regions of the items fpos_ + k*64 + lane (the first e are real; the others get a region
        // in range).  jlo_ is the region of the first item; one_ says every item lies in it.
        auto f_regions = [&](auto full, uint32_t fpos_, uint32_t e, uint32_t jlo_, bool one_, uint32_t (&reg)[V]) {
            constexpr bool FULL = decltype(full)::value;
            const uint32_t *key = BYTES ? SX : VT;
            const uint32_t last = fpos_ + e - 1u;   // position of the ensemble's last item
            if (one_) {
#pragma unroll
                for (int k = 0; k < V; ++k) reg[k] = jlo_;
            } else {
                // the next eight region starts, read at once (lane q: start jlo_ + 1 + q)
                const uint32_t jq = jlo_ + 1u + t;
                const uint32_t ks = (t < 8u && jq < nb) ? key[jq] : 0xFFFFFFFFu;
                if (__builtin_amdgcn_readlane(ks, 7) > last) {
                    // at most seven of them inside the ensemble: a uniform pass over them, each
                    // lane counting the starts at or before its item (equal starts, i.e. empty
                    // regions, all count)
#pragma unroll
                    for (int k = 0; k < V; ++k) reg[k] = jlo_;
                    const uint32_t nin = (uint32_t)__popcll(__ballot(ks <= last));   // a prefix of the lanes
                    for (uint32_t q = 0; q < nin; ++q) {
                        const uint32_t st = __builtin_amdgcn_readlane(ks, q);
#pragma unroll
                        for (int k = 0; k < V; ++k) reg[k] += fpos_ + (uint32_t)k * 64u + t >= st ? 1u : 0u;
                    }
                } else {
                    // many short regions: a binary search per lane
#pragma unroll
                    for (int k = 0; k < V; ++k) {
                        const uint32_t i = (uint32_t)k * 64u + t;
                        jlo_ = f_region(fpos_ + (FULL || i < e ? i : 0u), jlo_);   // positions grow with k
                        reg[k] = jlo_;
                    }
                }
            }
        };
        // The first stage on item i = k*64 + lane of an ensemble at fpos_: whether it passes,
        // the value it carries on, and the hash kind's child count.  x is the element (u32
        // kinds); j the item's region, ls_/lv_ its line's address and position (text).
        // text: bytes from the staging window (staged) or by buffer loads (the output-count pass)
        auto f_item = [&](auto staged, uint32_t i, bool act, uint32_t fpos_, uint32_t x, uint32_t j, uint32_t thr,
                          uint32_t ls_, uint32_t lv_, uint32_t &item, uint32_t &aux) -> bool {
            aux = 0;
            if constexpr (!BYTES) {
                item = x;
                bool kp;
                if constexpr (KIND == RS_MODFILTER) {
                    kp = mod_pow2 ? ((x & (modm - 1u)) == modr) : (x % modm == modr);
                } else if constexpr (HASHK) {
                    const uint32_t h = fmix32(x ^ salt_key(0));
                    kp = h & 1u;
                    aux = (h >> 1) & 3u;
                } else {
                    kp = x < (WALK ? CX[j] : thr);
                }
                return act && kp;
            } else {
                // signal: the line's address plus the line-relative position; tag: the address
                const uint32_t ls = TAG ? SX[j] : ls_;
                const uint32_t adr = TAG ? fpos_ + i : ls_ + (fpos_ - lv_) + i;
                item = adr;
                const bool in_line = act && (!TAG || adr < ls + (VT[j + 1] - VT[j]));
                const bool at_start = adr == ls;
                uint32_t cb, pb;
                if constexpr (decltype(staged)::value) {
                    const uint8_t *tw = (const uint8_t *)fsl;
                    const uint32_t ix = in_line ? adr - tsbase : 0u;
                    cb = tw[ix];
                    pb = tw[ix ? ix - 1u : 0u];
                } else {
                    cb = __builtin_amdgcn_raw_buffer_load_b8(rtext, in_line ? adr : 0u, 0, 0);
                    pb = __builtin_amdgcn_raw_buffer_load_b8(rtext, adr - (at_start ? 0u : 1u), 0, 0);
                }
                const uint32_t prev = at_start ? 32u : pb;
                return in_line && cb != 32u && prev == 32u;
            }
        };
        bool failed = false;
        bool out_ok = true;   // the claim's output base is known (ordered output stream)
        // ---- ordered output stream: count this claim's outputs, then learn its base from the
        // claims before it (decoupled look-back over the stream's claims) before producing.
        unsigned long long out_rank = 0;
        if (a.emit_outputs) {
            uint32_t fpos = vbeg, fj = 0, jlo = 0;
            bool fdone = WALK ? (vbeg >= vend) : (nb == 0);
            unsigned long long n_out = 0;
            while (!fdone) {
                const uint32_t rend = WALK ? vend : uni(VT[fj + 1]);
                const uint32_t e = min(EW, rend - fpos);
                if (e) {
                    const uint32_t ls = BYTES ? uni(SX[fj]) : 0u, lv = BYTES ? uni(VT[fj]) : 0u;
                    const uint32_t thr = (CTXP && !WALK) ? uni(CX[fj]) : 0u;
                    uint32_t reg[V], x[V];
                    if constexpr (WALK) f_regions(BoolC<false>{}, fpos, e, jlo, false, reg);
                    if constexpr (!BYTES) load_ens(fpos, e, x);
#pragma unroll
                    for (int k = 0; k < V; ++k) {
                        const uint32_t i = (uint32_t)k * 64u + t;
                        uint32_t item, aux;
                        const uint32_t j = WALK ? reg[k] : fj;
                        const bool keep = f_item(BoolC<false>{}, i, i < e, fpos, BYTES ? 0u : x[k], j, thr, ls, lv, item, aux);
                        const uint32_t nout = keep ? (HASHK ? aux : 1u) : 0u;
                        n_out += (uint32_t)__popcll(__ballot(nout & 1u)) + 2u * (uint32_t)__popcll(__ballot(nout & 2u));
                    }
                    if constexpr (WALK) {
                        const uint32_t kl = (e - 1u) >> 6, ll = (e - 1u) & 63u;
#pragma unroll
                        for (int k = 0; k < V; ++k)
                            if ((uint32_t)k == kl) jlo = __builtin_amdgcn_readlane(reg[k], ll);
                    }
                }
                fpos += e;
                if constexpr (WALK) {
                    fdone = (fpos == vend);
                } else if (fpos == rend) {
                    ++fj;
                    fdone = (fj == nb);
                }
            }
            // look-back: words are (epoch tag << 40) | (flag << 38) | value, flag 1 = this claim's
            // own count, flag 2 = inclusive prefix through this claim, flag 3 = no valid prefix
            // (a predecessor's look-back gave up).  The whole wave looks back 64 claims per step:
            // lane q reads claim base - 1 - q, and the step ends at the nearest claim holding flag
            // 2 or 3, summing the counts before it (a wave reduction).  A step waits while any claim
            // it needs has published nothing; each wait is bounded in real time (s_memrealtime
            // counts at 100 MHz): past the bound the claim publishes flag 3, writes no outputs and
            // raises the launch's error flag, so every wave still finishes and the host reports a
            // device error instead of waiting for ever.
            unsigned long long prefix = 0;
            uint32_t lb_ok = 1;
            {
                GLOBAL unsigned long long *lb = sd.lookback;
                const unsigned long long tagw = (unsigned long long)epoch_tag << 40;
                const unsigned long long mask38 = (1ull << 38) - 1ull;
                const unsigned long long limit = 100ull * a.lb_wait_us;
                if (t == 0)
                    __hip_atomic_store(&lb[cidx], tagw | (1ull << 38) | (n_out & mask38), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                uint32_t base = cidx;   // the claims before base are still to be accounted for
                unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
                while (base > 0u) {
                    const bool valid = t < base;
                    const unsigned long long w =
                        valid ? __hip_atomic_load(&lb[base - 1u - t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
                    const uint32_t fl = (valid && (w >> 40) == (unsigned long long)epoch_tag) ? (uint32_t)(w >> 38) & 3u : 0u;
                    const uint64_t stop = __ballot(fl >= 2u);
                    // lanes [0, need) take part: up to the nearest flag 2 or 3, else every valid lane
                    const uint32_t need = stop ? (uint32_t)__builtin_ctzll(stop) + 1u : min(base, 64u);
                    const uint64_t needm = need >= 64u ? ~0ull : (1ull << need) - 1ull;
                    if (__ballot(fl == 0u) & needm) {   // a claim it needs has published nothing yet
                        if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
                            lb_ok = 0;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(2);
                        continue;
                    }
                    if (stop && __builtin_amdgcn_readlane(fl, need - 1u) == 3u) {
                        lb_ok = 0;
                        break;
                    }
                    prefix += wave_sum_u64(t < need ? (w & mask38) : 0ull);
                    if (stop) break;
                    base = base > 64u ? base - 64u : 0u;
                    t0 = __builtin_amdgcn_s_memrealtime();
                }
                // the outputs must fit the stream's output array (k_max items per element)
                const unsigned long long cap = (unsigned long long)sd.n_elements * KE;
                if (prefix + n_out > cap) lb_ok = 0;
                if (t == 0) {
                    __hip_atomic_store(&lb[cidx],
                                       lb_ok ? tagw | (2ull << 38) | ((prefix + n_out) & mask38) : tagw | (3ull << 38),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (!lb_ok) __hip_atomic_fetch_or(&ctl[CTL_ERROR], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            out_rank = ((unsigned long long)uni((uint32_t)(prefix >> 32)) << 32) | uni((uint32_t)prefix);
            lb_ok = uni(lb_ok);
            if (!lb_ok) out_rank = 0;
            out_ok = lb_ok != 0u;
        }
        GLOBAL uint32_t *const out_items = out_ok ? sd.out_items : nullptr;

        // ---- node state (all uniform)
        uint32_t h1 = 0, t1 = 0, h2 = 0, t2 = 0;            // data queue heads and tails
        uint32_t h2w = 0, t2w = 0;                          // their slots in the second queue
        uint32_t sh1 = 0, st1 = 0, sh2 = 0, st2 = 0;        // signal queue heads and tails
        uint32_t sq1 = 0, sq2 = 0;                          // signal queues (entry n in lane n mod 64)
        // enumerating node: signal strategy walks region fj at position fpos;
        // tag strategy walks ensembles of EW consecutive positions from fpos.
        // (text under tags starts at the word boundary below: its firings take aligned words)
        uint32_t fj = 0, fpos = (BYTES && TAG) ? (vbeg & ~3u) : vbeg, jlo = 0;
        uint32_t rend = 0, ls = 0, lv = 0;                  // current region's end, line address, line position
        // tag strategy: start of region jlo + 1 (every position below it lies in region jlo or before)
        uint32_t jnext = 0xFFFFFFFFu;
        if constexpr (WALK) {
            if (nb > 1u) jnext = uni((BYTES ? SX : VT)[1]);
        }
        if constexpr (!WALK) {
            if (nb) {
                rend = uni(VT[1]);
                if constexpr (BYTES) ls = uni(SX[0]);
            }
        }
        // lane-resolved signals: the next region whose end the enumerating node has not signalled,
        // and that end
        uint32_t jb = 0;
        uint32_t bnext = 0;
        if constexpr (LANES) {
            if (nb) bnext = uni(VT[1]);
        }
        // lane-resolved signals finish once every position is enumerated and every region's end
        // is signalled (empty regions included)
        bool fdone = LANES ? (vbeg >= vend && nb == 0) : TAG ? (vbeg >= vend) : (nb == 0);
        uint32_t ej = 0;                      // signal strategy: region E is in
        uint32_t ja = 0, a_items = 0;         // signal strategy: region A closes next, items it has taken
        Acc acc;
        acc_reset(acc);
        uint32_t utag = 0;                    // tag strategy: region every lane's accumulator belongs to
        // lane n counts statistic n of this claim: firings, items, full firings and signals per node
        uint32_t stv = 0;
        const bool collect = a.collect_stats != 0u;
        auto stat = [&](uint32_t n, uint32_t v) {
            if (collect) stv += (t == n) ? v : 0u;
        };
        // every scheduler iteration fires a node; a claim needs at most a few firings per
        // element and per region, so this bound only trips on a scheduling error
        const uint32_t iter_cap =
            (uint32_t)min(8ull * ((unsigned long long)(vend - vbeg) + nb) + 64ull, 0xFFFFFFFFull);
        uint32_t iters = 0;

        if (spos != fpos) stage(fpos);
        if constexpr (BYTES && TAG) {
            tr_f0 = fpos;
            tr_m = 0xFFFFFFFFu;
            tring_request(0u);
        }

        // tree: the second sink's per-lane accumulators (the filter's survivors) and their region
        uint32_t k2c = 0, k2r = 0;
        unsigned long long k2s = 0;
        auto flush2 = [&]() {   // per lane, into the region's slots (LDS atomics)
            if constexpr (TREE) {
                if (k2c) {
                    atomicAdd(&s_kcnt[k2r], k2c);
                    atomicAdd(&s_ksum[k2r], k2s);
                }
                k2c = 0;
                k2s = 0;
            }
        };
        // the second sink takes survivor x of region j (per lane)
        auto sink2 = [&](bool keep, uint32_t x, uint32_t j) {
            if constexpr (TREE) {
                if (keep) {
                    if (j != k2r) {
                        flush2();
                        k2r = j;
                    }
                    k2c += 1u;
                    k2s += (unsigned long long)x;
                }
            }
        };

        // per-lane flush of the accumulator into region slot j (LDS atomics)
        auto flush_lane = [&](uint32_t j) {
            if (acc.cnt) {
                atomicAdd(&s_cnt[j], acc.cnt);
                atomicAdd(&s_sum[j], acc.sum);
                atomicMin(&s_min[j], acc.mn);
                atomicMax(&s_max[j], acc.mx);
            }
            acc_reset(acc);
        };
        // whole-wave flush of accumulators that all belong to region j
        auto flush_wave = [&](uint32_t j) {
            const Acc r = wave_reduce(acc);
            if (t == 0 && r.cnt) {
                // one lane of the wave that owns this LDS: a plain read-modify-write (the wave's
                // LDS accesses take effect in program order, after any lane's atomics before it)
                s_cnt[j] += r.cnt;
                s_sum[j] += r.sum;
                s_min[j] = min(s_min[j], r.mn);
                s_max[j] = max(s_max[j], r.mx);
            }
            acc_reset(acc);
        };

        // ---------------- A: the aggregating node, one firing of e items from its queue head
        auto a_fire = [&](auto full, uint32_t e) {
            constexpr bool FULL = decltype(full)::value;
            const uint32_t hw = HAS_E ? h2w : (h1 & (D1 - 1u));   // head slot
            const uint32_t *qv = HAS_E ? q2v : q1v;
            const uint8_t *qt = HAS_E ? q2t : q1t;
            uint32_t y[V], tg[V];
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const uint32_t pos = qslot(DA, hw, (uint32_t)k * 64u + t);
                y[k] = qv[pos];
                if constexpr (TAGQ) tg[k] = qt[pos]; else tg[k] = 0u;
            }
            if constexpr (LANES) {
                // each lane's region: the head region ja plus the pending signals at or before its
                // item (a signal at queue position p ends a region just before the item at p)
                const uint32_t sqa = HAS_E ? sq2 : sq1, sha = HAS_E ? sh2 : sh1;
                const uint32_t pend = (HAS_E ? st2 : st1) - sha, hq = HAS_E ? h2 : h1;
                const uint32_t ns =
                    (uint32_t)__popcll(__ballot(((t - sha) & (SQ - 1u)) < pend && sqa - hq < e));
#pragma unroll
                for (int k = 0; k < V; ++k) tg[k] = ja;
                for (uint32_t q = 0; q < ns; ++q) {
                    const uint32_t p = __builtin_amdgcn_readlane(sqa, (sha + q) & (SQ - 1u)) - hq;
#pragma unroll
                    for (int k = 0; k < V; ++k) tg[k] += (uint32_t)k * 64u + t >= p ? 1u : 0u;
                }
            }
            uint32_t tf = 0, tl = 0;
            if constexpr (PERLANE) {
                // regions of the ensemble's first and last items
                tf = uni(tg[0]);
                const uint32_t kl = (e - 1u) >> 6, ll = (e - 1u) & 63u;
#pragma unroll
                for (int k = 0; k < V; ++k)
                    if ((uint32_t)k == kl) tl = __builtin_amdgcn_readlane(tg[k], ll);
            }
#pragma unroll
            for (int k = 0; k < V; ++k) {
                // the expansion's children arrive as pre-images x ^ K(j+1); finishing the hash
                // here completes H(x, j+1)
                if constexpr (HASHK) y[k] = fmix32(y[k]);
            }
            if (out_items) {
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const uint32_t i = (uint32_t)k * 64u + t;
                    if (FULL || i < e) out_items[out_rank + i] = y[k];   // serial order
                }
            }
            if (!PERLANE || tf == tl) {
                if constexpr (PERLANE) {
                    if (tf != utag) {   // every lane's accumulator closes together
                        flush_wave(utag);
                        utag = tf;
                    }
                }
#pragma unroll
                for (int k = 0; k < V; ++k) acc_add(acc, y[k], FULL || (uint32_t)k * 64u + t < e);
            } else if (tl - tf < 8u && (tl - tf + 1u) * 16u <= e) {
                // the ensemble spans a few regions of many items each: one wave reduction per
                // region that ends in it, whose total one lane adds to the region's slot (per-lane
                // flushes would pile onto the same slot); the last region stays open in the
                // accumulators
                if (tf != utag) {
                    flush_wave(utag);
                    utag = tf;
                }
                for (uint32_t r = tf; r < tl; ++r) {
#pragma unroll
                    for (int k = 0; k < V; ++k) acc_add(acc, y[k], (FULL || (uint32_t)k * 64u + t < e) && tg[k] == r);
                    flush_wave(r);
                }
#pragma unroll
                for (int k = 0; k < V; ++k) acc_add(acc, y[k], (FULL || (uint32_t)k * 64u + t < e) && tg[k] == tl);
                utag = tl;
            } else if (!TAGQ || (tl - tf + 1u) * 8u > e) {
                // regions of a few items each: each lane flushes where its own items change region
                // (tags grow along the queue), then every lane flushes at the end
                uint32_t lt = utag;
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const bool act = FULL || (uint32_t)k * 64u + t < e;
                    if (act && tg[k] != lt) {
                        flush_lane(lt);
                        lt = tg[k];
                    }
                    acc_add(acc, y[k], act);
                }
                flush_lane(lt);
                utag = tl;
            } else {
                // tags, many regions of 8 or more items on average: round by round, the lanes of
                // one region inside each 8-lane block fold into that region's last lane in the
                // block (a segmented scan over DPP row shifts), which alone adds to the region's
                // slot; lanes of one region would otherwise serialise on the slot's atomics
                if (__ballot(acc.cnt != 0u)) flush_wave(utag);   // what the accumulators hold
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const bool act = FULL || (uint32_t)k * 64u + t < e;
                    const uint32_t key = act ? tg[k] : 0xFFFFFFFFu;   // no region has this key
                    // every lane reads its neighbours' keys before any lane-dependent test: a DPP
                    // read under a partial exec mask sees disabled source lanes as out of range
                    const uint32_t k1 = dpp_or<0x111, 0xF>(0xFFFFFFFEu, key);   // row_shr:1
                    const uint32_t k2 = dpp_or<0x112, 0xF>(0xFFFFFFFEu, key);   // row_shr:2
                    const uint32_t k4 = dpp_or<0x114, 0xF>(0xFFFFFFFEu, key);   // row_shr:4
                    const uint32_t kn = dpp_or<0x101, 0xF>(0xFFFFFFFFu, key);   // row_shl:1
                    const uint32_t b = t & 7u;
                    const bool t1 = (b >= 1u) & (k1 == key), t2 = (b >= 2u) & (k2 == key),
                               t4 = (b >= 4u) & (k4 == key);
                    // the block's last lane of a region: the block ends, or the next lane's key differs
                    const bool lead = act & ((b == 7u) | (kn != key));
                    const uint32_t c = seg_scan32<0>(act ? 1u : 0u, t1, t2, t4);
                    if (lead) atomicAdd(&s_cnt[key], c);
                    const unsigned long long sm = seg_sum64(act ? y[k] : 0u, t1, t2, t4);
                    if (lead) atomicAdd(&s_sum[key], sm);
                    const uint32_t mn = seg_scan32<1>(act ? y[k] : 0xFFFFFFFFu, t1, t2, t4);
                    if (lead) atomicMin(&s_min[key], mn);
                    const uint32_t mx = seg_scan32<2>(act ? y[k] : 0u, t1, t2, t4);
                    if (lead) atomicMax(&s_max[key], mx);
                }
                utag = tl;
            }
            if constexpr (LANES) {
                // the signals at or before the new head end their regions now
                uint32_t &sha = HAS_E ? sh2 : sh1;
                const uint32_t sqa = HAS_E ? sq2 : sq1;
                const uint32_t pend = (HAS_E ? st2 : st1) - sha, hq = HAS_E ? h2 : h1;
                const uint32_t nc =
                    (uint32_t)__popcll(__ballot(((t - sha) & (SQ - 1u)) < pend && sqa - hq <= e));
                ja += nc;
                sha += nc;
                stat(ST_SIGNALS + 2, nc);
            }
            if constexpr (HAS_E) {
                h2 += e;
                h2w = qslot(D2, h2w, e);
            } else {
                h1 += e;
            }
            a_items += e;
            out_rank += e;
            stat(ST_FIRINGS + 2, 1u);
            stat(ST_ITEMS + 2, e);
            if constexpr (FULL) stat(ST_FULL + 2, 1u);
        };

        // ---------------- E: the second node, one firing of e items from q1's head
        auto e_fire = [&](auto full, uint32_t e) {
            constexpr bool FULL = decltype(full)::value;
            uint32_t x[V], c[V], tg[V];
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const uint32_t pos = (h1 + (uint32_t)k * 64u + t) & (D1 - 1u);
                x[k] = q1v[pos];
                if constexpr (HASHK) c[k] = q1a[pos]; else c[k] = 1u;
                if constexpr (TAGQ) tg[k] = q1t[pos]; else tg[k] = 0u;
            }
            // output counts of every round (they do not depend on the word lengths below)
            uint64_t b0[V], b1[V];
            uint32_t total = 0;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const bool act = FULL || (uint32_t)k * 64u + t < e;
                const uint32_t nout = act ? c[k] : 0u;
                b0[k] = __ballot(nout & 1u);
                b1[k] = KE == 3u ? __ballot(nout & 2u) : 0ull;
                total += (uint32_t)__popcll(b0[k]) + 2u * (uint32_t)__popcll(b1[k]);
            }
            if constexpr (BYTES) {
                // word length: the run of non-space bytes from the word's start, within its line.
                // Every round's first window (the 16 bytes from the aligned word holding the start)
                // is requested before any round is examined, so their round trips overlap; a word
                // that reaches past its window goes on 32 bytes at a time.  Loads are range-checked
                // word by word (bytes past the array read as zero, which is not a space, and the
                // line's end bounds the run anyway).
                uint32_t wv[V][4];
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const bool act = FULL || (uint32_t)k * 64u + t < e;
                    const uint32_t q = act ? (x[k] & ~3u) : 0u;
#pragma unroll
                    for (int d = 0; d < 4; ++d) wv[k][d] = __builtin_amdgcn_raw_buffer_load_b32(rtext, q + 4u * d, 0, 0);
                }
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    if (!(FULL || (uint32_t)k * 64u + t < e)) continue;
                    const uint32_t j = TAGQ ? tg[k] : ej;
                    const uint32_t le = SX[j] + (VT[j + 1] - VT[j]);
                    const uint32_t p = x[k];
                    const uint32_t a = p & 3u;
                    uint64_t lo = (uint64_t)space_bytes(wv[k][0]) | ((uint64_t)space_bytes(wv[k][1]) << 32);
                    uint64_t hi = (uint64_t)space_bytes(wv[k][2]) | ((uint64_t)space_bytes(wv[k][3]) << 32);
                    if (a) {   // drop the bytes before the start
                        lo = (lo >> (8u * a)) | (hi << (64u - 8u * a));
                        hi >>= 8u * a;
                    }
                    const uint32_t win = 16u - a;   // bytes of the window from the start
                    uint32_t len = lo ? ((uint32_t)__builtin_ctzll(lo) >> 3) : hi ? 8u + ((uint32_t)__builtin_ctzll(hi) >> 3) : win;
                    if (len == win && le - p > win) {
                        // the word reaches past the window
                        uint32_t q = p + win;   // aligned
                        for (;;) {
                            uint32_t m[8];
#pragma unroll
                            for (int d = 0; d < 8; ++d) m[d] = space_bytes(__builtin_amdgcn_raw_buffer_load_b32(rtext, q + 4u * d, 0, 0));
                            uint32_t step = 32u;
#pragma unroll
                            for (int d = 7; d >= 0; --d)
                                if (m[d]) step = 4u * (uint32_t)d + ((uint32_t)__builtin_ctz(m[d]) >> 3);
                            len += step;
                            q += 32u;
                            if (step < 32u || p + len >= le) break;
                        }
                    }
                    x[k] = min(len, le - p);
                }
            }
            // The firing takes the longest prefix of the ensemble whose outputs fit the free
            // slots (the scheduler guarantees room for the first item's worst case); offsets are
            // exclusive prefixes in ensemble order, so the items that fit form a prefix.  When the
            // whole ensemble's outputs fit (the usual case) no item needs the room test.
            const uint32_t room = D2 - (t2 - h2);
            uint32_t taken = 0, made = 0;
            auto write_rounds = [&](auto fit_all) {
                constexpr bool FIT = decltype(fit_all)::value;
                uint32_t run = 0;
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const bool act = FULL || (uint32_t)k * 64u + t < e;
                    const uint32_t nout = act ? c[k] : 0u;
                    uint32_t within = rank_below(b0[k]);
                    if constexpr (KE == 3u) within += 2u * rank_below(b1[k]);
                    const uint32_t off = run + within;
                    const uint32_t slot0 = qslot(D2, t2w, off);   // first child's slot
                    uint64_t fits = 0;
                    if constexpr (!FIT) {
                        fits = __ballot(act && off + nout <= room);
                        taken += (uint32_t)__popcll(fits);
                        made += (uint32_t)__popcll(b0[k] & fits) + 2u * (uint32_t)__popcll(b1[k] & fits);
                    }
#pragma unroll
                    for (uint32_t ch = 0; ch < KE; ++ch) {
                        const uint32_t sl = ch == 0u ? slot0 : qslot(D2, slot0, ch);
                        const uint64_t m = FIT ? __ballot(ch < nout) : (__ballot(ch < nout) & fits);
                        const uint32_t pos = pick(m, sl, D2 + t);
                        // child ch of x leaves as its pre-image x ^ K(ch+1) (hash kind); a word as its length
                        q2v[pos] = HASHK ? x[k] ^ salt_key(ch + 1u) : x[k];
                        if constexpr (TAGQ) q2t[pos] = (uint8_t)tg[k];
                    }
                    run += (uint32_t)__popcll(b0[k]) + 2u * (uint32_t)__popcll(b1[k]);
                }
                if constexpr (FIT) {
                    taken = e;
                    made = total;
                }
            };
            if (total <= room) write_rounds(BoolC<true>{}); else write_rounds(BoolC<false>{});
            if constexpr (LANES) {
                // the signals at or before the last item taken pass to the second signal queue,
                // each re-based to the outputs of the items before it (the scheduler sized the
                // ensemble so that they fit; equal positions beyond the room stay behind)
                const uint32_t pend = st1 - sh1, free2 = SQ - (st2 - sh2);
                const uint32_t rel = sq1 - h1;
                const bool fw = ((t - sh1) & (SQ - 1u)) < pend && rel <= taken;
                const uint32_t nf = min((uint32_t)__popcll(__ballot(fw)), free2);
                if (nf) {
                    const uint32_t r = fw ? rel : 0u;
                    const uint32_t np = t2 + bits_below<V>(b0, r) + 2u * bits_below<V>(b1, r);
                    // S1 entry sh1 + i becomes S2 entry st2 + i
                    const uint32_t i = (t - st2) & (SQ - 1u);
                    const uint32_t moved = (uint32_t)__shfl((int)np, (int)((sh1 + i) & (SQ - 1u)), 64);
                    sq2 = i < nf ? moved : sq2;
                    st2 += nf;
                    sh1 += nf;
                    stat(ST_SIGNALS + 1, nf);
                }
            }
            h1 += taken;
            t2 += made;
            t2w = qslot(D2, t2w, made);
            stat(ST_FIRINGS + 1, 1u);
            stat(ST_ITEMS + 1, taken);
            stat(ST_FULL + 1, taken == EW ? 1u : 0u);
        };

        // ---------------- F: the enumerating node, one firing of e items from fpos
        // nbound (lane-resolved signals): the ends of regions jb .. jb + nbound - 1 fall in this
        // ensemble or at its end, and their signals go out with it
        // Text under tags, four bytes per lane.  The firing's ensemble [fpos, fpos + e) starts at
        // a multiple of 4 on this path; lane t of round k takes the aligned word at
        // a = fpos + 4 (64 k + t) from the staged window and flags its bytes four at a time: a byte
        // starts a word when it lies in a line, is not a space, and follows a space or is its
        // line's first byte.  A word holds at most two starts (each follows a space or a line
        // start), queued with their lines' tags in address order.  The lines that meet the
        // ensemble are those from jlo on that start at or before its last byte: lane q reads line
        // jlo + q's start and end once, and every lane then walks them as uniform values (no
        // chain of LDS round trips).  jlo becomes the last of them.  Returns how many it queued.
        auto text_starts4 = [&](uint32_t e) -> uint32_t {
            constexpr uint32_t NW = EW / 4u, RW = (NW + 63u) / 64u;
            const uint32_t last = fpos + e - 1u;
            uint32_t inl[RW], lst[RW], rof[RW];
#pragma unroll
            for (uint32_t k = 0; k < RW; ++k) inl[k] = lst[k] = rof[k] = 0u;
            for (uint32_t jb0 = jlo;;) {
                const uint32_t jq = jb0 + t;
                const bool have = jq < nb;
                const uint32_t cs = have ? SX[jq] : 0xFFFFFFFFu;
                const uint32_t ce = have ? cs + (VT[jq + 1u] - VT[jq]) : 0u;
                const uint32_t nd = (uint32_t)__popcll(__ballot(have && cs <= last));   // a prefix of the lanes
                for (uint32_t d = 0; d < nd; ++d) {
                    const uint32_t st = __builtin_amdgcn_readlane(cs, d), en = __builtin_amdgcn_readlane(ce, d);
#pragma unroll
                    for (uint32_t k = 0; k < RW; ++k) {
                        const uint32_t a = fpos + 4u * (k * 64u + t);
                        const uint32_t sb = st - a;   // the line's first byte in this word when below 4
                        const uint32_t lo = st > a ? min(sb, 4u) : 0u;
                        const uint32_t hi = en > a ? min(en - a, 4u) : 0u;
                        // bytes lo .. hi - 1 of the word lie in line jb0 + d
                        const uint32_t m = hi > lo ? (0x80808080u >> (8u * (4u - hi))) & (0x80808080u << (8u * lo)) : 0u;
                        inl[k] |= m;
                        rof[k] |= (m >> 7) * (jb0 + d);
                        lst[k] |= (sb < 4u && m != 0u) ? 0x80u << (8u * sb) : 0u;
                    }
                }
                if (nd < 64u) {
                    if (nd) jlo = jb0 + nd - 1u;
                    break;
                }
                jb0 += 64u;
            }
            uint32_t run = 0;
#pragma unroll
            for (uint32_t k = 0; k < RW; ++k) {
                const uint32_t i = k * 64u + t;
                const uint32_t a = fpos + 4u * i;
                const uint32_t nin = (i < NW && 4u * i < e) ? min(4u, e - 4u * i) : 0u;   // bytes of the ensemble
                const uint32_t ens = nin >= 4u ? 0x80808080u : 0x80808080u & ((1u << (8u * nin)) - 1u);
                const uint32_t off = a - (tr_f0 + tr_m * TWB);   // the word's byte offset in its window
                const uint32_t wi = (tr_m & 1u) * (TWB / 4u) + (nin ? off >> 2 : 1u);
                const uint32_t cur = fsl[wi];
                const uint32_t prv = (nin && off == 0u) ? tr_carry : fsl[wi - 1u];
                const uint32_t sp = space_bytes(cur);
                const uint32_t after_sp = (sp << 8) | (space_bytes(prv) >> 24);
                const uint32_t starts = ~sp & (after_sp | lst[k]) & inl[k] & ens;
                const uint32_t c = (uint32_t)__builtin_popcount(starts);   // 0, 1 or 2
                const uint32_t f0 = starts ? (uint32_t)__builtin_ctz(starts) >> 3 : 0u;
                const uint32_t s1 = starts & (starts - 1u);
                const uint32_t f1 = s1 ? (uint32_t)__builtin_ctz(s1) >> 3 : 0u;
                const uint64_t b1 = __ballot(c & 1u), b2 = __ballot(c & 2u);
                const uint32_t within = rank_below(b1) + 2u * rank_below(b2);
                const uint32_t pc = (uint32_t)__popcll(b1) + 2u * (uint32_t)__popcll(b2);
                const uint32_t spill = D1 + ((t1 + run + pc + t - within) & 63u);
                const uint32_t p0 = pick(__ballot(c != 0u), (t1 + run + within) & (D1 - 1u), spill);
                const uint32_t p1 = pick(b2, (t1 + run + within + 1u) & (D1 - 1u), spill);
                q1v[p0] = a + f0;
                q1t[p0] = (uint8_t)(rof[k] >> (8u * f0));
                q1v[p1] = a + f1;
                q1t[p1] = (uint8_t)(rof[k] >> (8u * f1));
                run += pc;
            }
            return run;
        };
        auto f_node = [&](auto full, uint32_t e, uint32_t nbound) {
            constexpr bool FULL = decltype(full)::value;
            // the items' own regions: for tags, and for lane-resolved signals of a kind that reads
            // the parent's context
            constexpr bool FREG = TAG || (LANES && (CTXP || TREE));
            constexpr bool SWAR = BYTES && TAG;   // text under tags: four bytes per lane
            bool one = true;
            if constexpr (FREG) one = jnext > fpos + e - 1u;
            uint32_t reg[V], x[V];
            uint64_t kb[V];   // kept-item masks per round (lane-resolved signals)
            if constexpr (SWAR) {
#pragma unroll
                for (int k = 0; k < V; ++k) reg[k] = 0;
            } else if constexpr (FREG) {
                f_regions(full, fpos, e, jlo, one, reg);
            } else {
#pragma unroll
                for (int k = 0; k < V; ++k) reg[k] = fj;
            }
            if constexpr (!BYTES) {
                if (spos != fpos) stage(fpos);
                wait_vmem<0>();   // the slot's copy has landed
#pragma unroll
                for (int k = 0; k < V; ++k) x[k] = fsl[k * 64 + t];
                // the slot's words are in registers: request the next firing's ensemble now, so that
                // its copy overlaps this firing too
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
                stage(fpos + e);
            } else if constexpr (SWAR) {
                const uint32_t m = (fpos - tr_f0) / TWB;
                if (m != tr_m) {
                    wait_vmem<0>();   // window m has landed
                    // the word before window m, read before its buffer is refilled
                    tr_carry = m ? uni(fsl[((m - 1u) & 1u) * (TWB / 4u) + TWB / 4u - 1u]) : 0x20202020u;
                    tr_m = m;
                    tring_request(m + 1u);
                }
            } else {
                const uint32_t adr0 = TAG ? fpos : ls + (fpos - lv);   // the firing's first byte
                if (tspos != adr0) stage_text(adr0);
                wait_vmem<0>();   // the window has landed
#pragma unroll
                for (int k = 0; k < V; ++k) x[k] = 0;
            }
            const uint32_t thr = (CTXP && !WALK) ? uni(CX[fj]) : 0u;
            uint32_t run = 0;
            if constexpr (SWAR) run = text_starts4(e);   // also moves jlo to the last line it met
#pragma unroll
            for (int k = 0; k < (SWAR ? 0 : V); ++k) {
                const uint32_t i = (uint32_t)k * 64u + t;
                uint32_t item, aux;
                const bool keep = f_item(BoolC<true>{}, i, FULL || i < e, fpos, x[k], reg[k], thr, ls, lv, item, aux);
                sink2(keep, x[k], reg[k]);   // the tree's second child of the filter
                const uint64_t b = __ballot(keep);
                kb[k] = b;
                const uint32_t within = rank_below(b), pc = (uint32_t)__popcll(b);
                // dropped lanes write spill slots on the banks the kept ones leave free
                const uint32_t pos = pick(b, (t1 + run + within) & (D1 - 1u), D1 + ((t1 + run + pc + t - within) & 63u));
                q1v[pos] = item;
                if constexpr (HASHK) q1a[pos] = (uint8_t)aux;
                if constexpr (TAGQ) q1t[pos] = (uint8_t)reg[k];
                run += pc;
            }
            if constexpr (FREG) {
                if (!one) {
                    if constexpr (!SWAR) {
                        const uint32_t kl = (e - 1u) >> 6, ll = (e - 1u) & 63u;
#pragma unroll
                        for (int k = 0; k < V; ++k)
                            if ((uint32_t)k == kl) jlo = __builtin_amdgcn_readlane(reg[k], ll);
                    }
                    jnext = jlo + 1u < nb ? uni((BYTES ? SX : VT)[jlo + 1u]) : 0xFFFFFFFFu;
                }
            }
            if constexpr (LANES) {
                if (nbound) {
                    // each region end's signal sits at the queue position of the first kept item
                    // after it; lane i mod 64 holds signal-queue entry i
                    const uint32_t i = (t - st1) & (SQ - 1u);
                    const bool mine = i < nbound;
                    const uint32_t rel = mine ? min(VT[min(jb + i + 1u, nb)] - fpos, e) : 0u;
                    const uint32_t p = t1 + bits_below<V>(kb, rel);
                    sq1 = mine ? p : sq1;
                    st1 += nbound;
                    jb += nbound;
                    stat(ST_SIGNALS + 0, nbound);
                }
            }
            if constexpr (!BYTES) {
                // requested above, once the slot's words were in registers
            } else {
                // the next firing's window: the rest of this line, else the next line (tags: the next
                // address); a wrong guess is staged again when that firing starts
                const uint32_t nf = fpos + e;
                uint32_t nadr = 0xFFFFFFFFu;
                if constexpr (TAG) {
                    (void)nf;   // the window ring requests ahead by itself
                } else {
                    if (nf < rend) nadr = ls + (nf - lv);
                    else if (fj + 1u < nb) nadr = uni(SX[fj + 1u]);
                }
                if (nadr != 0xFFFFFFFFu) stage_text(nadr);
            }
            t1 += run;
            fpos += e;
            stat(ST_FIRINGS + 0, 1u);
            stat(ST_ITEMS + 0, e);
            if constexpr (FULL) stat(ST_FULL + 0, 1u);
        };

        // ---------------- fused firings (hash kind)
        // A full ensemble that lies inside one region, met while the first queue and both signal
        // queues are empty, needs neither a tag per item nor a signal to keep regions apart: F and
        // E fire on it as one firing, each survivor writing its children straight into A's queue
        // in serial order (no compaction of survivors into the first queue, no second read of
        // them), and A then takes every whole 64-lane round of its queue.  During a run of such
        // firings A's queue is a plain array from slot 0, its leftover of under 64 items moved to
        // the front after each firing; the first queue's storage, empty meanwhile, is a second
        // staging slot, so the next ensemble's copy is in flight while one is processed.  A region
        // that ends between two ensembles closes as its end signal would close it: A takes the
        // leftover (the signal's credit) and ends the region.  The run stops at the first ensemble
        // that is not full or spans a region end, leaving the state the scheduler expects.
        uint32_t spos2 = 0xFFFFFFFFu;   // position whose ensemble the second slot holds or receives
        // region containing position pos (< vend), searching up from region j0 (start <= pos)
        auto region_of = [&](uint32_t pos, uint32_t j0) -> uint32_t {
            uint32_t r = j0;
            while (uni(VT[r + 1u]) <= pos) ++r;
            return r;
        };
        // whether the ensemble at fpos is full and inside one region
        auto fuse_ok = [&]() -> bool {
            if constexpr (!WALK) {
                return fpos + EW <= rend;
            } else {
                if (fpos + EW > vend) return false;
                const uint32_t r = region_of(fpos, TAG ? jlo : jb);
                return uni(VT[r + 1u]) >= fpos + EW;
            }
        };
        // A takes the n (< 64) items at the front of its queue: the last items of a region
        auto fuse_drain = [&](uint32_t n) {
            if (n) {
                const uint32_t y = fmix32(q2v[t]);
                if (out_items && t < n) out_items[out_rank + t] = y;
                acc_add(acc, y, t < n);
                a_items += n;
                out_rank += n;
                h2 += n;
                stat(ST_FIRINGS + 2, 1u);
                stat(ST_ITEMS + 2, n);
            }
        };
        // A takes every whole 64-lane round of the avail items at the front of its queue (one
        // region's children), w items per firing; returns how many it took
        auto fuse_a = [&](uint32_t avail) -> uint32_t {
            uint32_t base = 0;
            while (avail - base >= EW) {
                uint32_t y[V];
#pragma unroll
                for (int k = 0; k < V; ++k) y[k] = fmix32(q2v[base + (uint32_t)k * 64u + t]);
                if (out_items) {
#pragma unroll
                    for (int k = 0; k < V; ++k) out_items[out_rank + (uint32_t)k * 64u + t] = y[k];
                }
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    acc.sum += (unsigned long long)y[k];
                    acc.mn = min(acc.mn, y[k]);
                    acc.mx = max(acc.mx, y[k]);
                }
                acc.cnt += (uint32_t)V;
                base += EW;
                out_rank += EW;
                stat(ST_FIRINGS + 2, 1u);
                stat(ST_ITEMS + 2, EW);
                stat(ST_FULL + 2, 1u);
            }
            const uint32_t nr = (avail - base) >> 6;   // whole rounds short of a full ensemble
            if (nr) {
                // every round's slot is read first (slots past the queue's end lie inside its
                // array and are not used), so the reads overlap
                uint32_t y[V > 1 ? V - 1 : 1];
#pragma unroll
                for (int k = 0; k + 1 < V; ++k) y[k] = q2v[base + (uint32_t)k * 64u + t];
#pragma unroll
                for (int k = 0; k + 1 < V; ++k) {
                    if ((uint32_t)k < nr) {
                        const uint32_t v = fmix32(y[k]);
                        if (out_items) out_items[out_rank + (uint32_t)k * 64u + t] = v;
                        acc.sum += (unsigned long long)v;
                        acc.mn = min(acc.mn, v);
                        acc.mx = max(acc.mx, v);
                    }
                }
                acc.cnt += nr;
                base += nr * 64u;
                out_rank += nr * 64u;
                stat(ST_FIRINGS + 2, 1u);
                stat(ST_ITEMS + 2, nr * 64u);
            }
            a_items += base;
            h2 += base;
            return base;
        };
        // F and E as one firing on the full ensemble in src (a staging slot): survivor x writes
        // its c children, as pre-images x ^ K(j+1), to A's queue from slot lt on, in serial
        // order; returns the new end of A's queue.  Each lane writes its three candidate slots
        // off+2, off+1, off in that order; a slot past a lane's last child belongs to a later
        // item of the firing, whose own (later) write of a smaller child index lands on it, or
        // lies past the firing's last child.  Lanes without children write their dump slots.
        auto fuse_fe = [&](auto counting, const uint32_t *src, uint32_t lt, uint32_t region) -> uint32_t {
            constexpr bool COUNT = decltype(counting)::value;   // E's item count for the statistics
            if constexpr (TREE) {   // the ensemble's survivors all belong to one region
                if (k2r != region) {
                    flush2();
                    k2r = region;
                }
            }
            uint32_t x[V];
#pragma unroll
            for (int k = 0; k < V; ++k) x[k] = src[k * 64 + (int)t];
            uint32_t run = lt, kept = 0;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                const uint32_t h = fmix32(x[k] ^ salt_key(0));
                // survivors (bit 0) with an odd child count (bit 1), and with two or three (bit 2)
                const uint64_t b0 = __ballot((h & 3u) == 3u);
                const uint64_t b1 = __ballot((h & 5u) == 5u);
                if constexpr (COUNT) kept += (uint32_t)__popcll(__ballot(h & 1u));
                if constexpr (TREE) {   // the tree's second child of the filter
                    k2c += h & 1u;
                    k2s += (unsigned long long)((h & 1u) ? x[k] : 0u);
                }
                const uint32_t off = run + rank_below(b0) + 2u * rank_below(b1);
                const uint32_t dst = pick(b0 | b1, off, FDUMP + t);
                q2v[dst + 2u] = x[k] ^ salt_key(3u);
                order();
                q2v[dst + 1u] = x[k] ^ salt_key(2u);
                order();
                q2v[dst] = x[k] ^ salt_key(1u);
                order();
                run += (uint32_t)__popcll(b0) + 2u * (uint32_t)__popcll(b1);
            }
            stat(ST_FIRINGS + 0, 1u);
            stat(ST_ITEMS + 0, EW);
            stat(ST_FULL + 0, 1u);
            stat(ST_FIRINGS + 1, 1u);
            stat(ST_ITEMS + 1, kept);
            return uni(run);
        };
        // tags and lane-resolved signals: the region of the ensemble at fpos (< vend); when it is not
        // the one A's accumulators hold, A takes the leftover lt of the old one and closes it (for
        // lane-resolved signals the region ends before fpos then count as signalled and taken).
        // Returns whether the ensemble is full and inside that region.
        auto fuse_walk_region = [&](uint32_t &lt) -> bool {
            // still inside the region A holds, as the cached start of the next region shows: no
            // region table read (the common case of a run inside a long region)
            if constexpr (LANES) {
                if (utag == jb && jb < nb && fpos + EW <= bnext) {
                    ja = jb;
                    return true;
                }
            } else {
                if (utag == jlo && fpos + EW <= jnext) return true;
            }
            const uint32_t r = region_of(fpos, TAG ? jlo : jb);
            if (r != utag) {
                fuse_drain(lt);
                lt = 0;
                flush_wave(utag);
                utag = r;
            }
            if constexpr (LANES) {
                if (r != jb) {
                    stat(ST_SIGNALS + 0, r - jb);
                    stat(ST_SIGNALS + 1, r - jb);
                    stat(ST_SIGNALS + 2, r - jb);
                    jb = r;
                    bnext = uni(VT[r + 1u]);
                }
                ja = r;
            } else {
                if (r != jlo) {
                    jlo = r;
                    jnext = r + 1u < nb ? uni(VT[r + 1u]) : 0xFFFFFFFFu;
                }
            }
            return uni(VT[r + 1u]) >= fpos + EW;
        };
        // a run of fused firings from fpos (the ensemble there is full and inside one region).  The
        // loop tests the next ensemble at its bottom: a test at its top, which the entry has
        // already passed, would give the loop a second entry.
        auto fuse_run = [&]() {
            // what A's queue holds (fewer than w items, none past a signal) goes first
            if (h2 != t2) a_fire(BoolC<false>{}, t2 - h2);
            h2w = t2w = 0;
            uint32_t lt = 0;   // items at the front of A's queue
            if constexpr (WALK) (void)fuse_walk_region(lt);
            if constexpr (HYB) {
                if (utag != fj) {
                    flush_wave(utag);
                    utag = fj;
                }
            }
            for (;;) {
                // ---- the ensemble's slot, and the next ensemble's copy into the other slot (both
                // slots' positions are updated by selects: a conditional store to one or the other
                // would be merged into a store through a selected address, which keeps them out
                // of registers)
                const bool in2 = spos2 == fpos;
                if (!in2 && spos != fpos) stage(fpos);
                const uint32_t nx = fpos + EW;
                const bool ahead = nx < vend;
                if (ahead)
                    lds_copy<V>(rsrc_words(elems + (size_t)nx * 4u, min(EW, vend - nx) * 4u),
                                uni(in2 ? lds_addr(fsl) : lds_addr(q1v)), t, vend - nx >= EW);
                const uint32_t npos = ahead ? nx : 0xFFFFFFFFu;
                spos = in2 ? npos : spos;
                spos2 = in2 ? spos2 : npos;
                if (ahead) wait_vmem<copy_ops<V>()>(); else wait_vmem<0>();
                // ---- F and E, then A on every whole round
                const uint32_t *src = in2 ? q1v : fsl;
                const uint32_t reg = WALK ? utag : fj;   // the ensemble's region
                const uint32_t nt =
                    collect ? fuse_fe(BoolC<true>{}, src, lt, reg) : fuse_fe(BoolC<false>{}, src, lt, reg);
                t2 += nt - lt;
                fpos += EW;
                const uint32_t used = fuse_a(nt);
                lt = nt - used;
                if (lt && used) {   // the leftover to the front
                    const uint32_t v = q2v[used + t];
                    order();
                    if (t < lt) q2v[t] = v;
                    order();
                }
                // ---- region ends at fpos, and whether the next ensemble can be fused
                if constexpr (!WALK) {
                    if (fpos == rend) {
                        // region ja ends: A takes the items before its signal, then ends it
                        // (per-stage choice: the items are tagged, and A closes the region it holds)
                        fuse_drain(lt);
                        lt = 0;
                        if constexpr (HYB) {
                            flush_wave(utag);
                        } else if (a_items) {
                            const Acc r = wave_reduce(acc);
                            if (t == 0) {
                                s_cnt[ja] = r.cnt;
                                s_sum[ja] = r.sum;
                                s_min[ja] = r.mn;
                                s_max[ja] = r.mx;
                            }
                            acc_reset(acc);
                            a_items = 0;
                        }
                        // the region's signal, and those of the empty regions after it
                        do {
                            ++fj;
                            ++ej;
                            ++ja;
                            if constexpr (!HYB) {
                                stat(ST_SIGNALS + 0, 1u);
                                stat(ST_SIGNALS + 1, 1u);
                                stat(ST_SIGNALS + 2, 1u);
                            }
                        } while (fj < nb && uni(VT[fj + 1u]) == fpos);
                        fdone = fj == nb;   // (an unconditional store, as for the slots above)
                        if (fdone) break;
                        rend = uni(VT[fj + 1u]);
                        if constexpr (HYB) utag = fj;
                    }
                    if (fpos + EW > rend) break;
                } else {
                    if (fpos + EW > vend) break;
                    if (!fuse_walk_region(lt)) break;
                }
            }
            // A's queue holds the leftover in slots [0, lt) for the scheduler
            t2w = lt;
            if constexpr (TAGQ) {
                if (t < lt) q2t[t] = (uint8_t)utag;
            }
            if constexpr (TAG) {
                fdone = (fpos == vend);
            } else if constexpr (LANES) {
                fdone = (fpos == vend && jb == nb);
            }
            if (spos2 != 0xFFFFFFFFu) {   // no copy into the first queue's storage outlives the run
                wait_vmem<0>();
                spos2 = 0xFFFFFFFFu;
            }
        };

        for (;;) {
            if (++iters > iter_cap) {
                failed = true;
                break;
            }
            // ---------------- A (drains first)
            {
                const uint32_t hq = HAS_E ? h2 : h1, tq = HAS_E ? t2 : t1;
                uint32_t e = 0;
                bool fire = false;
                if constexpr (LANES) {
                    // signals with no item before them end their regions at once
                    uint32_t &sh = HAS_E ? sh2 : sh1;
                    const uint32_t pend = (HAS_E ? st2 : st1) - sh;
                    const uint32_t nh = (uint32_t)__popcll(
                        __ballot(((t - sh) & (SQ - 1u)) < pend && (HAS_E ? sq2 : sq1) == hq));
                    if (nh) {
                        ja += nh;
                        sh += nh;
                        stat(ST_SIGNALS + 2, nh);
                        continue;
                    }
                }
                if constexpr (SIGQ) {
                    uint32_t &sh = HAS_E ? sh2 : sh1;
                    const uint32_t stq = HAS_E ? st2 : st1;
                    if (sh < stq) {
                        const uint32_t p = __builtin_amdgcn_readlane(HAS_E ? sq2 : sq1, sh & (SQ - 1u));
                        if (p == hq) {
                            // signal phase: no item precedes the signal, so region ja ends here
                            if (a_items) {
                                const Acc r = wave_reduce(acc);
                                if (t == 0) {
                                    s_cnt[ja] = r.cnt;
                                    s_sum[ja] = r.sum;
                                    s_min[ja] = r.mn;
                                    s_max[ja] = r.mx;
                                }
                                acc_reset(acc);
                                a_items = 0;
                            }
                            ++ja;
                            ++sh;
                            stat(ST_SIGNALS + 2, 1u);
                            continue;
                        }
                        e = min(p - hq, EW);   // the signal's credit bounds the ensemble
                        fire = true;
                    }
                }
                if (!fire) {
                    const bool up_done = HAS_E ? (fdone && h1 == t1) : fdone;
                    const uint32_t n = tq - hq;
                    // lane-resolved signals: a full signal queue makes A fire what it has
                    const bool sq_full = LANES && (HAS_E ? st2 - sh2 : st1 - sh1) == SQ;
                    if (n >= EW || ((up_done || sq_full) && n > 0)) {
                        e = min(n, EW);
                        fire = true;
                    }
                }
                if (fire) {
                    if (e == EW) a_fire(BoolC<true>{}, e); else a_fire(BoolC<false>{}, e);
                    continue;
                }
            }
            // ---------------- E
            if constexpr (HAS_E) {
                // E may fire when the first item's worst-case output fits; the firing itself
                // keeps only the prefix whose actual outputs fit
                const bool room = D2 - (t2 - h2) >= KE;
                uint32_t e = 0;
                bool sig = false, pending = false;
                if constexpr (LANES) {
                    pending = true;   // e is decided here
                    const uint32_t pend = st1 - sh1, free2 = SQ - (st2 - sh2);
                    // signals with no item before them pass on at once (sender rule: S2 has room)
                    const uint32_t nh = min(
                        (uint32_t)__popcll(__ballot(((t - sh1) & (SQ - 1u)) < pend && sq1 == h1)), free2);
                    if (nh) {
                        const uint32_t i = (t - st2) & (SQ - 1u);
                        sq2 = i < nh ? t2 : sq2;
                        st2 += nh;
                        sh1 += nh;
                        stat(ST_SIGNALS + 1, nh);
                        continue;
                    }
                    const uint32_t n = t1 - h1;
                    // a full first signal queue makes E fire what it has
                    if (room && free2 && n && (n >= EW || fdone || pend == SQ)) {
                        e = min(n, EW);
                        // at most free2 signals can pass on: the first that cannot bounds the ensemble
                        const uint32_t nle = (uint32_t)__popcll(
                            __ballot(((t - sh1) & (SQ - 1u)) < pend && sq1 - h1 <= e));
                        if (nle > free2) e = __builtin_amdgcn_readlane(sq1, (sh1 + free2) & (SQ - 1u)) - h1;
                    }
                }
                if constexpr (SIGQ) {
                    if (sh1 < st1) {
                        pending = true;
                        const uint32_t p = __builtin_amdgcn_readlane(sq1, sh1 & (SQ - 1u));
                        if (p == h1) sig = true; else if (room) e = min(p - h1, EW);
                    }
                }
                if (sig) {
                    if (st2 - sh2 < SQ) {   // forward the signal (sender rule: S2 has room)
                        sq2 = t == (st2 & (SQ - 1u)) ? t2 : sq2;
                        ++st2;
                        ++sh1;
                        ++ej;
                        stat(ST_SIGNALS + 1, 1u);
                        continue;
                    }
                } else {
                    if (!pending) {
                        const uint32_t n = t1 - h1;
                        if (room && (n >= EW || (fdone && n > 0))) e = min(n, EW);
                    }
                    if (e) {
                        if (e == EW) e_fire(BoolC<true>{}, e); else e_fire(BoolC<false>{}, e);
                        continue;
                    }
                }
            }
            // ---------------- F and E fused, then A (hash kind, a full ensemble inside one region)
            if constexpr (FUSE) {
                if (!fdone && h1 == t1 && sh1 == st1 && sh2 == st2 && fuse_ok()) {
                    fuse_run();
                    // the queue state after the run is opaque to the compiler: threading what it
                    // knows of it into the next pass would merge the scheduler loop into the claim
                    // loop and shuffle its state at every join
                    asm volatile("" : "+s"(h1), "+s"(sh1), "+s"(sh2));
                    continue;
                }
            }
            // ---------------- F
            if constexpr (LANES) {
                if (!fdone) {
                    uint32_t e = min(EW, vend - fpos);
                    uint32_t nbound = 0;
                    // the next end not yet signalled (kept in a register): most firings of long
                    // regions hold none
                    if (jb < nb && bnext - fpos <= e) {
                        // region ends at or before fpos + e: lane q looks at region jb + q (ends
                        // grow with the region index, so the hits form a prefix)
                        const uint32_t jq = jb + t;
                        const bool in = jq < nb && VT[min(jq + 1u, nb)] - fpos <= e;
                        const uint32_t nall = (uint32_t)__popcll(__ballot(in));
                        nbound = min(nall, SQ - (st1 - sh1));
                        // the first end left unsignalled bounds the ensemble (sender rule: S1 has room)
                        if (jb + nbound < nb) {
                            const uint32_t nxt = uni(VT[jb + nbound + 1u]) - fpos;
                            e = min(e, nxt);
                        }
                    }
                    // room for every item (all might pass)
                    if ((e || nbound) && D1 - (t1 - h1) >= e) {
                        if (e == EW) {
                            f_node(BoolC<true>{}, e, nbound);
                        } else if (e) {
                            f_node(BoolC<false>{}, e, nbound);
                        } else {   // ends with no item before them: signals only
                            const uint32_t i = (t - st1) & (SQ - 1u);
                            sq1 = i < nbound ? t1 : sq1;
                            st1 += nbound;
                            jb += nbound;
                            stat(ST_SIGNALS + 0, nbound);
                        }
                        fdone = (fpos == vend && jb == nb);
                        if (nbound && jb < nb) bnext = uni(VT[jb + 1u]);
                        continue;
                    }
                }
            } else if (!fdone) {
                const uint32_t lim = TAG ? vend : rend;
                const uint32_t e = min(EW, lim - fpos);
                const bool ends = !TAG && fpos + e == rend;
                // room for every item (all might pass) and, at a region's end, for its signal (the
                // per-stage choice tags instead)
                if (D1 - (t1 - h1) >= e && (!ends || HYB || st1 - sh1 < SQ)) {
                    if (e == EW) f_node(BoolC<true>{}, e, 0u);
                    else if (e) f_node(BoolC<false>{}, e, 0u);
                    if constexpr (TAG) {
                        fdone = (fpos == vend);
                    } else if (ends) {
                        if constexpr (!HYB) {
                            sq1 = t == (st1 & (SQ - 1u)) ? t1 : sq1;
                            ++st1;
                            stat(ST_SIGNALS + 0, 1u);
                        }
                        ++fj;
                        fdone = (fj == nb);
                        if (!fdone) {
                            rend = uni(VT[fj + 1]);
                            if constexpr (BYTES) {
                                ls = uni(SX[fj]);
                                lv = uni(VT[fj]);
                            }
                        }
                    }
                    continue;
                }
            }
            // nothing fireable
            if (fdone && h1 == t1 && h2 == t2 && sh1 == st1 && sh2 == st2) break;
            failed = true;   // cannot happen: some node is always fireable (Lemma 2)
            break;
        }

        if constexpr (PERLANE) flush_wave(utag);
        flush2();
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // no staged copy outlives the claim
        order();
        if (failed && t == 0) __hip_atomic_fetch_or(&ctl[CTL_ERROR], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

        // ---- end(): one record per parent, written once
        {
            const SDesc se = load_sdesc(sdl);   // read here, after the scheduler loop
            for (uint32_t i = t; i < nb; i += 64u) {
                const uint32_t p = p0 + i;
                if (a.agg_fields & RS_COUNT) se.agg_count[p] = s_cnt[i];
                if (a.agg_fields & RS_SUM) se.agg_sum[p] = s_sum[i];
                if (a.agg_fields & RS_MIN) se.agg_min[p] = s_min[i];
                if (a.agg_fields & RS_MAX) se.agg_max[p] = s_max[i];
                if constexpr (TREE) {
                    if (a.agg_fields & RS_KEPT_COUNT) se.agg_kcount[p] = s_kcnt[i];
                    if (a.agg_fields & RS_KEPT_SUM) se.agg_ksum[p] = s_ksum[i];
                }
            }
            if (a.collect_stats && t < ST_SIGNALS + 3 && stv)
                __hip_atomic_fetch_add(&se.stats[t], (unsigned long long)stv, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
        order();
        g = g1;
        g1 = g_next;
        cur = nxt;
        // the next claim's first ensemble, when its range lies inside its element array (a
        // malformed claim is caught before any of its own reads).  Requested after the copy of the
        // next claim's region table above, which waits for that table's loads and would wait for
        // this copy too if it came first.
        pf_g = 0xFFFFFFFFu;
        if constexpr (!BYTES) {
            if (g < a.total_claims) {
                const uint32_t nnb = cur.nb;
                const uint32_t vb = uni(__builtin_amdgcn_readlane(cur.off[0], 0));
                uint32_t ve = 0;
#pragma unroll
                for (uint32_t q = 0; q < R; ++q)
                    if (q == (nnb >> 6)) ve = uni(__builtin_amdgcn_readlane(cur.off[q], nnb & 63u));
                if (vb < ve && ve <= cur.n_elements) {
                    lds_copy<V>(rsrc_words(cur.elements + (size_t)vb * 4u, min(EW, ve - vb) * 4u), uni(lds_addr(fsl)),
                                t, ve - vb >= EW);
                    pf_g = g;
                }
            }
        }
    }
}

// ---------------------------------------------------------------- launch table

using KernelFn = void (*)(LaunchArgs);

// Ensemble width w = 64 * V: one wave, V items per lane per firing.
template <int KIND, int STRAT>
static KernelFn pick_width(uint32_t w) {
    switch (w) {
        case 64: return rs_pipeline<KIND, STRAT, 1>;
        case 128: return rs_pipeline<KIND, STRAT, 2>;
        case 256: return rs_pipeline<KIND, STRAT, 4>;
        case 512: return rs_pipeline<KIND, STRAT, 8>;
        case 1024: return rs_pipeline<KIND, STRAT, 16>;
        default: return nullptr;
    }
}

// Lane-resolved signals: u32 kinds, w up to 256.
template <int KIND>
static KernelFn pick_lanes(uint32_t w) {
    if constexpr (KIND == RS_TEXT_WORDS) {
        return nullptr;
    } else {
        switch (w) {
            case 64: return rs_pipeline<KIND, RS_SIGNAL_LANES, 1>;
            case 128: return rs_pipeline<KIND, RS_SIGNAL_LANES, 2>;
            case 256: return rs_pipeline<KIND, RS_SIGNAL_LANES, 4>;
            default: return nullptr;
        }
    }
}

// Enumeration with tags downstream (the per-stage choice): kinds with a second stage.
template <int KIND>
static KernelFn pick_enum_tag(uint32_t w) {
    if constexpr (KIND == RS_HASH_EXPAND || KIND == RS_HASH_TREE || KIND == RS_TEXT_WORDS) {
        return pick_width<KIND, RS_ENUM_TAG>(w);
    } else {
        return nullptr;
    }
}

template <int KIND>
static KernelFn pick_strategy(uint32_t s, uint32_t w) {
    switch (s) {
        case RS_TAG: return pick_width<KIND, RS_TAG>(w);
        case RS_SIGNAL: return pick_width<KIND, RS_SIGNAL>(w);
        case RS_SIGNAL_LANES: return pick_lanes<KIND>(w);
        case RS_ENUM_TAG: return pick_enum_tag<KIND>(w);
        default: return nullptr;
    }
}

static KernelFn pick(uint32_t kind, uint32_t s, uint32_t w) {
    switch (kind) {
        case RS_MODFILTER: return pick_strategy<RS_MODFILTER>(s, w);
        case RS_HASH_EXPAND: return pick_strategy<RS_HASH_EXPAND>(s, w);
        case RS_TEXT_WORDS: return pick_strategy<RS_TEXT_WORDS>(s, w);
        case RS_GRAPH_THRESH: return pick_strategy<RS_GRAPH_THRESH>(s, w);
        case RS_HASH_TREE: return pick_strategy<RS_HASH_TREE>(s, w);
        default: return nullptr;
    }
}

uint32_t lanes_of(uint32_t ensemble_width) { return ensemble_width ? 64u : 0u; }

uint32_t dyn_lds_bytes(uint32_t kind, uint32_t strategy, uint32_t width, uint32_t qdepth, uint32_t bmax) {
    return dyn_layout(kind, strategy, width, qdepth, bmax).bytes;
}

// ---------------------------------------------------------------- HBM probe

// Plain copy, 16 bytes per lane per step, grid-stride: the achievable-bandwidth reference
// for the pipeline kernels and the known-size copy that calibrates traffic counters.
__global__ void __launch_bounds__(256) probe_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                  unsigned long long n16) {
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

int launch_probe_copy(const void *src, void *dst, unsigned long long bytes, uint32_t n_cu, void *stream) {
    hipLaunchKernelGGL(probe_copy, dim3(n_cu * 4), dim3(256), 0, (hipStream_t)stream, (const uint4 *)src,
                       (uint4 *)dst, bytes / 16);
    return (int)hipGetLastError();
}

// ---------------------------------------------------------------- no-allocation scratch

static_assert(CTL_WORDS * 4u == NOALLOC_TABLE_OFF, "control block fills the scratch's first part");
static_assert(sizeof(StreamDev) <= NOALLOC_TABLE_STRIDE && sizeof(NoallocTable) <= 4096u,
              "table fits its part and a kernel argument");

// Device state of the no-allocation entry point: control block, stream table, statistics.  Each
// device holds its own copy until the process ends; calls on one device share it.  Host code
// never uses this name as an address: it is looked up per device below.
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

int noalloc_scratch(void **out) {
    static std::mutex mu;
    static void *addr[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    if (dev < 0 || dev >= 64) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // the current device's copy
        if (e != hipSuccess) return (int)e;
        addr[dev] = p;
    }
    *out = addr[dev];
    return (int)hipSuccess;
}

// Clears the control block and the statistics words, then writes the stream table (a kernel, not
// a memset or a copy from host memory, so that the call allocates nothing and can be captured).
__global__ void __launch_bounds__(64) rs_noalloc_init(uint8_t *base, NoallocTable tab) {
    const uint32_t t = threadIdx.x;
    uint32_t *ctl = (uint32_t *)(base + NOALLOC_CTL_OFF);
    for (uint32_t i = t; i < CTL_WORDS; i += 64u) ctl[i] = 0u;
    unsigned long long *st = (unsigned long long *)(base + NOALLOC_STATS_OFF);
    for (uint32_t i = t; i < NOALLOC_MAX_STREAMS * ST_WORDS; i += 64u) st[i] = 0ull;
    uint32_t *dst = (uint32_t *)(base + NOALLOC_TABLE_OFF);
    const uint32_t *src = (const uint32_t *)tab.s;
    for (uint32_t i = t; i < tab.n * (uint32_t)(sizeof(StreamDev) / 4u); i += 64u) dst[i] = src[i];
}

int launch_noalloc_init(void *base, const NoallocTable &tab, void *stream) {
    hipLaunchKernelGGL(rs_noalloc_init, dim3(1), dim3(64), 0, (hipStream_t)stream, (uint8_t *)base, tab);
    return (int)hipGetLastError();
}

bool kernel_supported(uint32_t kind, uint32_t strategy, uint32_t width) {
    return pick(kind, strategy, width) != nullptr;
}

// Prepares the control block for the launch that follows it on the same stream: claim
// counters to zero, and a new epoch for the look-back words.  A separate kernel (not a
// memset) so that a captured graph replays it correctly.
__global__ void __launch_bounds__(64) rs_reset(uint32_t *ctl) {
    const uint32_t t = threadIdx.x;
    if (t < CTL_NPART) ctl[CTL_PART + t * CTL_PART_STRIDE] = 0u;
    static_assert(CTL_NPART <= 64, "one lane per claim counter");
    if (t == 0) ctl[CTL_EPOCH] += 1u;
}

int launch_pipeline(uint32_t kind, uint32_t strategy, uint32_t width, const LaunchArgs &a, uint32_t grid,
                    void *stream, void *ev_begin, void *ev_end) {
    KernelFn k = pick(kind, strategy, width);
    if (!k) return (int)hipErrorInvalidValue;
    const hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(rs_reset, dim3(1), dim3(64), 0, st, a.ctl);
    hipError_t e = hipSuccess;
    if (ev_begin && (e = hipEventRecord((hipEvent_t)ev_begin, st)) != hipSuccess) return (int)e;
    hipLaunchKernelGGL(k, dim3(grid), dim3(lanes_of(width)), dyn_lds_bytes(kind, strategy, width, a.qdepth, a.bmax), st,
                       a);
    if ((e = hipGetLastError()) != hipSuccess) return (int)e;
    if (ev_end && (e = hipEventRecord((hipEvent_t)ev_end, st)) != hipSuccess) return (int)e;
    return (int)hipSuccess;
}

int blocks_per_cu(uint32_t kind, uint32_t strategy, uint32_t width, uint32_t qdepth, uint32_t bmax) {
    KernelFn k = pick(kind, strategy, width);
    if (!k) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, (int)lanes_of(width),
                                                    dyn_lds_bytes(kind, strategy, width, qdepth, bmax)) !=
        hipSuccess)
        return 0;
    return n;
}

}  // namespace rs
