// gfx950 kernels of the region-stateful streaming pipeline.
//
// One workgroup of W lanes is one SIMD processor in the sense of §2.2: it runs a
// whole pipeline instance (enumerating node F, optional second node E, aggregating
// node A) with a non-preemptive scheduler, and it competes with every other
// workgroup for parent batches ("claims") through a device atomic on a common
// counter, returning only when every claim of every stream in the launch is done.
// A firing of a node consumes an ensemble of at most w = W*V items: item i of the
// ensemble sits on lane i mod W, in round i / W, so one firing is V rounds of
// W-wide SIMD work.
//
// Nodes are joined by fixed-size LDS queues.  Data-dependent output counts are
// compacted with wave64 ballot/mbcnt ranks plus an LDS prefix over the waves.
// Region boundaries travel either
//   - as signals (RS_SIGNAL): an end-of-region slot sits in the data queue at its
//     exact stream position and a small signal queue records where the slots are;
//     the items between two slots are that signal's credit (the in-band form of the
//     credit protocol of §3.1), a consumer's ensemble never extends past the next
//     slot (the SIMD rule of §3.3), and a node consumes a slot only when no item
//     precedes it, running end() for that region; or
//   - as tags (RS_TAG): every queued item carries its region index, ensembles mix
//     regions freely, and the aggregating node reduces by tag (§5).
// Aggregates are exact integer reductions kept in LDS slots per claim and written
// once per parent; a claim always holds whole regions, so no aggregate is ever
// shared between workgroups.
//
// Elements reach the enumerating node through an LDS ring filled by direct
// global->LDS loads (global_load_lds_dwordx4), NS chunks deep, independent of
// where ensembles or regions begin; the next claim's region table is loaded into
// registers while the current claim runs.  The compiler does not track which chunk
// a read touches, so the ring is read with inline-asm ds_read and completion is
// managed with explicit vmcnt waits and a barrier that does not drain vmcnt.
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// ---------------------------------------------------------------- wave / workgroup helpers

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Workgroup barrier that waits for this wave's LDS operations only (not for
// outstanding global->LDS chunk loads, whose completion is waited for explicitly).
__device__ __forceinline__ void bar() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Wait until at most N vector-memory operations of this wave are outstanding.
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

__device__ __forceinline__ void wait_vm_n(uint32_t n) {
    switch (n) {
        case 0: wait_vm<0>(); break;
        case 1: wait_vm<1>(); break;
        case 2: wait_vm<2>(); break;
        case 3: wait_vm<3>(); break;
        case 4: wait_vm<4>(); break;
        case 5: wait_vm<5>(); break;
        case 6: wait_vm<6>(); break;
        default: wait_vm<7>(); break;
    }
}

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;

__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}

// Reads of the element ring, hidden from the compiler's wait insertion.
__device__ __forceinline__ uint32_t ring_u32(uint32_t addr) {
    uint32_t v;
    asm volatile("ds_read_b32 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(addr) : "memory");
    return v;
}
__device__ __forceinline__ void ring_u32x4(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t &v0,
                                           uint32_t &v1, uint32_t &v2, uint32_t &v3) {
    asm volatile(
        "ds_read_b32 %0, %4\n\t"
        "ds_read_b32 %1, %5\n\t"
        "ds_read_b32 %2, %6\n\t"
        "ds_read_b32 %3, %7\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(v0), "=&v"(v1), "=&v"(v2), "=&v"(v3)
        : "v"(a0), "v"(a1), "v"(a2), "v"(a3)
        : "memory");
}
__device__ __forceinline__ void ring_u32x2(uint32_t a0, uint32_t a1, uint32_t &v0, uint32_t &v1) {
    asm volatile(
        "ds_read_b32 %0, %2\n\t"
        "ds_read_b32 %1, %3\n\t"
        "s_waitcnt lgkmcnt(0)"
        : "=&v"(v0), "=&v"(v1)
        : "v"(a0), "v"(a1)
        : "memory");
}
__device__ __forceinline__ uint32_t ring_u8(uint32_t addr) {
    uint32_t v;
    asm volatile("ds_read_u8 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(addr) : "memory");
    return v;
}
__device__ __forceinline__ void ring_w8(uint32_t addr, uint32_t v) {
    asm volatile("ds_write_b8 %0, %1\n\ts_waitcnt lgkmcnt(0)" : : "v"(addr), "v"(v) : "memory");
}

// N ring bytes at the given LDS addresses, issued together and waited for once, all in
// one asm statement (no output register may be touched before the wait).
template <int N>
__device__ __forceinline__ void ring_read_u8(const uint32_t (&a)[N], uint32_t (&o)[N]) {
    if constexpr (N == 8) {
        asm volatile(
            "ds_read_u8 %0, %8\n\tds_read_u8 %1, %9\n\tds_read_u8 %2, %10\n\tds_read_u8 %3, %11\n\t"
            "ds_read_u8 %4, %12\n\tds_read_u8 %5, %13\n\tds_read_u8 %6, %14\n\tds_read_u8 %7, %15\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3]), "=&v"(o[4]), "=&v"(o[5]), "=&v"(o[6]),
              "=&v"(o[7])
            : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3]), "v"(a[4]), "v"(a[5]), "v"(a[6]), "v"(a[7])
            : "memory");
    } else if constexpr (N == 4) {
        asm volatile(
            "ds_read_u8 %0, %4\n\tds_read_u8 %1, %5\n\tds_read_u8 %2, %6\n\tds_read_u8 %3, %7\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(o[0]), "=&v"(o[1]), "=&v"(o[2]), "=&v"(o[3])
            : "v"(a[0]), "v"(a[1]), "v"(a[2]), "v"(a[3])
            : "memory");
    } else if constexpr (N == 2) {
        asm volatile("ds_read_u8 %0, %2\n\tds_read_u8 %1, %3\n\ts_waitcnt lgkmcnt(0)"
                     : "=&v"(o[0]), "=&v"(o[1])
                     : "v"(a[0]), "v"(a[1])
                     : "memory");
    } else {
#pragma unroll
        for (int k = 0; k < N; ++k) o[k] = ring_u8(a[k]);
    }
}

// V u32 ring words at the given LDS addresses, issued together, waited for once.
template <int V>
__device__ __forceinline__ void ring_read(const uint32_t (&addr)[V], uint32_t (&out)[V]) {
    if constexpr (V == 4) {
        ring_u32x4(addr[0], addr[1], addr[2], addr[3], out[0], out[1], out[2], out[3]);
    } else if constexpr (V == 2) {
        ring_u32x2(addr[0], addr[1], out[0], out[1]);
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) out[k] = ring_u32(addr[k]);
    }
}

// Exclusive prefix of per-item counts n[k] (0..3) over an ensemble laid out as item
// k*W + lane, in that order.  off[k] is the item's first output slot relative to the
// firing's base; total is the firing's output count (uniform).
template <int W, int V, bool TWO_BITS>
__device__ __forceinline__ void ens_scan(const uint32_t (&n)[V], uint32_t (&off)[V], uint32_t &total,
                                         uint32_t *scr) {
    constexpr uint32_t NW = W / 64;
    uint32_t within[V], wsum[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const uint64_t b0 = __ballot(n[k] & 1u);
        within[k] = rank_below(b0);
        wsum[k] = (uint32_t)__popcll(b0);
        if constexpr (TWO_BITS) {
            const uint64_t b1 = __ballot((n[k] >> 1) & 1u);
            within[k] += 2u * rank_below(b1);
            wsum[k] += 2u * (uint32_t)__popcll(b1);
        }
    }
    if constexpr (NW == 1) {
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            off[k] = run + within[k];
            run += wsum[k];
        }
        total = uni(run);
    } else {
        const uint32_t wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63u) == 0) {
#pragma unroll
            for (int k = 0; k < V; ++k) scr[k * NW + wv] = wsum[k];
        }
        bar();
        uint32_t run = 0;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            uint32_t before = 0, all = 0;
#pragma unroll
            for (uint32_t w = 0; w < NW; ++w) {
                const uint32_t s = scr[k * NW + w];
                before += (w < wv) ? s : 0u;
                all += s;
            }
            off[k] = run + before + within[k];
            run += all;
        }
        total = uni(run);
    }
}

// Exclusive prefix of arbitrary u32 values over the workgroup (one per lane).
template <int W>
__device__ __forceinline__ uint32_t wg_scan_u32(uint32_t v, uint32_t *scr, uint32_t &total) {
    const uint32_t ln = threadIdx.x & 63u;
    uint32_t inc = v;
#pragma unroll
    for (uint32_t o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o, 64);
        if (ln >= o) inc += u;
    }
    const uint32_t wsum = __shfl(inc, 63, 64);
    if constexpr (W == 64) {
        total = uni(wsum);
        return inc - v;
    } else {
        const uint32_t wv = threadIdx.x >> 6;
        if (ln == 63u) scr[wv] = wsum;
        bar();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (uint32_t i = 0; i < (uint32_t)W / 64u; ++i) {
            const uint32_t s = scr[i];
            before += (i < wv) ? s : 0u;
            all += s;
        }
        total = uni(all);
        return before + inc - v;
    }
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
__device__ __forceinline__ void acc_add(Acc &a, uint32_t y) {
    a.cnt += 1u;
    a.sum += (unsigned long long)y;
    a.mn = a.mn < y ? a.mn : y;
    a.mx = a.mx > y ? a.mx : y;
}

// Workgroup reduction of per-lane accumulators; every lane gets the result.
template <int W>
__device__ __forceinline__ Acc wg_reduce(Acc a, uint32_t *scr) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        a.cnt += __shfl_xor(a.cnt, o, 64);
        a.sum += __shfl_xor(a.sum, o, 64);
        const uint32_t m0 = __shfl_xor(a.mn, o, 64);
        const uint32_t m1 = __shfl_xor(a.mx, o, 64);
        a.mn = a.mn < m0 ? a.mn : m0;
        a.mx = a.mx > m1 ? a.mx : m1;
    }
    if constexpr (W == 64) {
        return a;
    } else {
        constexpr uint32_t NW = W / 64;
        const uint32_t wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63u) == 0) {
            scr[64 + wv] = a.cnt;
            scr[80 + 2 * wv] = (uint32_t)a.sum;
            scr[81 + 2 * wv] = (uint32_t)(a.sum >> 32);
            scr[112 + wv] = a.mn;
            scr[128 + wv] = a.mx;
        }
        bar();
        Acc r;
        acc_reset(r);
#pragma unroll
        for (uint32_t i = 0; i < NW; ++i) {
            r.cnt += scr[64 + i];
            r.sum += (unsigned long long)scr[80 + 2 * i] | ((unsigned long long)scr[81 + 2 * i] << 32);
            r.mn = r.mn < scr[112 + i] ? r.mn : scr[112 + i];
            r.mx = r.mx > scr[128 + i] ? r.mx : scr[128 + i];
        }
        return r;
    }
}

// ---------------------------------------------------------------- geometry

template <int W, int V, bool HAS_E>
struct Geo {
    static constexpr uint32_t EW = W * V;        // ensemble width: items one firing consumes
    static constexpr uint32_t R = 256 / W;       // region-table rows per lane
    static constexpr uint32_t BMAX = R * W - 1;  // parents in one claim, at most (B+1 offsets, R per lane)
    static constexpr uint32_t D1 = 2 * EW;       // data slots in front of the second node
    static constexpr uint32_t D2 = HAS_E ? 4 * EW : 1;   // in front of the third node (k = 3 expansion)
    static constexpr uint32_t SQ = 256;          // signal queue capacity (finite S of §3.1)
    static constexpr uint32_t CHB = 16 * W;      // bytes of one ring chunk: one 16-byte load per lane
    static constexpr uint32_t NS = W == 64 ? 8 : 4;   // chunks in the element ring
    static constexpr uint32_t RING = NS * CHB;
};

enum Misc : uint32_t {
    M_NEXT = 200, M_JLAST = 201, M_BASE_LO = 202, M_BASE_HI = 203, M_BAD = 204, M_WORDS = 208
};

// Region table of one claim, as loaded from HBM: lane t holds parents p0 + r*W + t, r < R.
template <int R>
struct ClaimRegs {
    uint32_t off[R];   // CSR offsets[p0 + i] (i <= nb), or start of region p0 + i (i < nb)
    uint32_t len[R];   // length of region p0 + i (start+length streams)
    uint32_t ctx[R];   // per-parent context
};

// ---------------------------------------------------------------- the pipeline kernel

template <int KIND, int STRAT, int W, int V>
__global__ void __launch_bounds__(W) rs_pipeline(LaunchArgs a) {
    constexpr bool TAG = (STRAT == RS_TAG);
    constexpr bool HAS_E = (KIND == RS_HASH_EXPAND || KIND == RS_TEXT_WORDS);
    constexpr bool BYTES = (KIND == RS_TEXT_WORDS);
    constexpr bool CTXP = (KIND == RS_GRAPH_THRESH);
    constexpr uint32_t EB = BYTES ? 1u : 4u;                       // element bytes
    constexpr uint32_t KE = (KIND == RS_HASH_EXPAND) ? 3u : 1u;    // outputs per input of E
    using G = Geo<W, V, HAS_E>;
    constexpr uint32_t EW = G::EW;

    __shared__ __attribute__((aligned(16))) uint8_t ring[G::RING];
    __shared__ uint32_t VT[G::BMAX + 1];             // region starts in enumeration order, end at [nb]
    __shared__ uint32_t SX[BYTES ? G::BMAX : 1];     // region start addresses (start+length streams)
    __shared__ uint32_t CX[CTXP ? G::BMAX : 1];      // per-parent context
    __shared__ uint32_t s_cnt[G::BMAX];
    __shared__ unsigned long long s_sum[G::BMAX];
    __shared__ uint32_t s_min[G::BMAX];
    __shared__ uint32_t s_max[G::BMAX];
    __shared__ uint32_t q1v[G::D1];
    __shared__ uint8_t q1a[KIND == RS_HASH_EXPAND ? G::D1 : 1];
    __shared__ uint16_t q1t[TAG ? G::D1 : 1];
    __shared__ uint32_t sp1[TAG ? 1 : G::SQ];
    __shared__ uint32_t q2v[G::D2];
    __shared__ uint16_t q2t[(HAS_E && TAG) ? G::D2 : 1];
    __shared__ uint32_t sp2[(HAS_E && !TAG) ? G::SQ : 1];
    __shared__ uint32_t misc[M_WORDS];

    const uint32_t t = threadIdx.x;
    const uint32_t wv = t >> 6;
    const uint32_t ring_base = lds_addr(ring);
    constexpr uint32_t R = G::R;
    // A single-wave processor needs no hardware barrier: a wave's LDS operations complete in
    // order, so only the compiler must be kept from moving memory accesses across this point.
    auto sync = [&]() {
        if constexpr (W == 64) asm volatile("" ::: "memory");
        else bar();
    };

    // stage parameters
    const uint32_t modm = a.param[0] ? a.param[0] : 4u;
    const uint32_t modr = a.param[1];
    const bool mod_pow2 = (modm & (modm - 1u)) == 0u;

    // launches completed so far, as a 24-bit tag in [1, 2^24 - 1] for the look-back words
    // (the control block only changes after every workgroup of a launch has finished)
    const uint32_t epoch_tag =
        uni(__hip_atomic_load(&a.ctl[CTL_EPOCH], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) % 0xFFFFFFu + 1u;

    // stream of global claim gg: the last with claim_begin <= gg
    auto stream_of = [&](uint32_t gg) -> uint32_t {
        uint32_t lo = 0, hi = a.n_streams;
        while (hi - lo > 1u) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.streams[mid].claim_begin <= gg) lo = mid; else hi = mid;
        }
        return lo;
    };
    // this lane's share of the region table of claim gg (loads only; consumed a claim later)
    auto load_claim = [&](uint32_t gg, ClaimRegs<R> &r) {
#pragma unroll
        for (uint32_t q = 0; q < R; ++q) r.off[q] = r.len[q] = r.ctx[q] = 0;
        if (gg >= a.total_claims) return;
        const StreamDev &sd = a.streams[stream_of(gg)];
        const uint32_t B = sd.parents_per_claim;
        const uint32_t p0 = (gg - sd.claim_begin) * B;
        const uint32_t nb = min(B, sd.n_parents - p0);
#pragma unroll
        for (uint32_t q = 0; q < R; ++q) {
            const uint32_t i = q * W + t;
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

    // claims are taken two ahead: g is worked on, g1 is next (its region table in registers)
    uint32_t first = 0, second = 0;
    if (t == 0) {
        first = atomicAdd(&a.ctl[CTL_CLAIM], 1u);
        second = atomicAdd(&a.ctl[CTL_CLAIM], 1u);
        misc[M_NEXT] = first;
        misc[M_NEXT + 1] = second;
    }
    sync();
    uint32_t g = uni(misc[M_NEXT]);
    uint32_t g1 = uni(misc[M_NEXT + 1]);
    ClaimRegs<R> cur;
    load_claim(g, cur);
    sync();

    while (g < a.total_claims) {
        uint32_t g_next = 0;
        if (t == 0) g_next = atomicAdd(&a.ctl[CTL_CLAIM], 1u);   // the claim after g1
        ClaimRegs<R> nxt;
        load_claim(g1, nxt);                                      // consumed at the next claim

        const StreamDev &sd = a.streams[stream_of(g)];
        const uint8_t *elems = (const uint8_t *)sd.elements;
        const uint32_t B = sd.parents_per_claim;
        const uint32_t cidx = g - sd.claim_begin;
        const uint32_t p0 = cidx * B;
        const uint32_t nb = uni(min(B, sd.n_parents - p0));
        const uint32_t nbytes_total = sd.n_elements * EB;

        // ---- region table of the claim (enumeration: findCount per parent)
        uint32_t vbeg, vend;
        if constexpr (!BYTES) {
#pragma unroll
            for (uint32_t q = 0; q < R; ++q) {
                const uint32_t i = q * W + t;
                if (i <= nb) VT[i] = cur.off[q];
                if constexpr (CTXP)
                    if (i < nb) CX[i] = cur.ctx[q];
            }
            sync();
            vbeg = uni(VT[0]);
            vend = uni(VT[nb]);
        } else {
            uint32_t carry = 0;
#pragma unroll
            for (uint32_t q = 0; q < R; ++q) {
                const uint32_t i = q * W + t;
                if (i < nb) SX[i] = cur.off[q];
                uint32_t tot;
                const uint32_t ex = wg_scan_u32<W>(i < nb ? cur.len[q] : 0u, misc, tot);
                if (i < nb) VT[i] = carry + ex;
                carry += tot;
                sync();
            }
            if (t == 0) VT[nb] = carry;
            sync();
            vbeg = 0;
            vend = carry;
        }
        for (uint32_t i = t; i < nb; i += W) {
            s_cnt[i] = 0;
            s_sum[i] = 0ull;
            s_min[i] = 0xFFFFFFFFu;
            s_max[i] = 0;
        }

        // The claim's regions must be ordered and inside the element array before any element
        // is read; a malformed stream is flagged and its claims are skipped.
        {
            bool bad = false;
            for (uint32_t i = t; i < nb; i += W) {
                if constexpr (!BYTES) {
                    bad |= (VT[i] > VT[i + 1]) || (i + 1u == nb && VT[nb] > sd.n_elements);
                } else {
                    const unsigned long long end = (unsigned long long)SX[i] + (VT[i + 1] - VT[i]);
                    const unsigned long long lim = (i + 1u < nb) ? SX[i + 1] : sd.n_elements;
                    bad |= end > lim;
                }
            }
            if (t == 0) misc[M_BAD] = 0;
            sync();
            if (bad) misc[M_BAD] = 1;
            sync();
            if (uni(misc[M_BAD])) {
                if (t == 0) {
                    atomicOr((unsigned int *)&sd.stats[ST_ERROR], 1u);
                    if (a.emit_outputs)   // successors of this claim must not wait for it
                        __hip_atomic_store(&sd.lookback[cidx], ((unsigned long long)epoch_tag << 40) | (2ull << 38),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    misc[M_NEXT] = g_next;
                }
                sync();
                g = g1;
                g1 = uni(misc[M_NEXT]);
                cur = nxt;
                continue;
            }
        }

        // ---- element ring: the claim's byte range, chunked from a 16-byte aligned base
        uint32_t b0, b1;
        if constexpr (!BYTES) {
            b0 = vbeg * 4u;
            b1 = vend * 4u;
        } else {
            b0 = nb ? uni(SX[0]) : 0u;
            b1 = nb ? uni(SX[nb - 1] + (VT[nb] - VT[nb - 1])) : 0u;
            if constexpr (TAG) {   // lines are enumerated over the claim's address range
                vbeg = b0;
                vend = b1;
            }
        }
        const uint32_t A0 = b0 & ~15u;
        const uint32_t nch = (b1 > b0) ? (b1 - A0 + G::CHB - 1u) / G::CHB : 0u;
        uint32_t ld_next = 0, ld_ready = 0;
        uint32_t partial_mask = 0;   // per lane: ring slots holding a partial tail block to patch

        auto issue = [&]() {
            const uint32_t c = ld_next;
            const uint32_t blk = A0 + c * G::CHB + t * 16u;
            const bool full = blk + 16u <= nbytes_total;
            const uint8_t *src = full ? elems + blk : (const uint8_t *)a.dummy;
            if (!full && blk < nbytes_total) partial_mask |= 1u << (c % G::NS);
            __builtin_amdgcn_global_load_lds((glb_void_t *)src,
                                             (lds_void_t *)(ring + (c % G::NS) * G::CHB + wv * 1024u), 16, 0, 0);
            ld_next = c + 1u;
        };
        // make chunks [0, k] readable
        auto ready_upto = [&](uint32_t k) {
            while (ld_ready <= k) {
                wait_vm_n(ld_next - 1u - ld_ready);
                if (partial_mask & (1u << (ld_ready % G::NS))) {
                    partial_mask &= ~(1u << (ld_ready % G::NS));
                    const uint32_t blk = A0 + ld_ready * G::CHB + t * 16u;
                    const uint32_t dst = ring_base + (ld_ready % G::NS) * G::CHB + t * 16u;
                    for (uint32_t k2 = 0; blk + k2 < nbytes_total; ++k2) ring_w8(dst + k2, elems[blk + k2]);
                }
                sync();
                ++ld_ready;
            }
        };
        // issue every chunk whose ring slot is free: chunk ld_next reuses the slot of
        // chunk ld_next - NS, which must end at or before need_from
        auto refill = [&](uint32_t need_from) {
            while (ld_next < nch && (ld_next < G::NS || A0 + (ld_next - G::NS + 1u) * G::CHB <= need_from)) issue();
        };
        auto ring_off = [&](uint32_t addr) -> uint32_t { return ring_base + ((addr - A0) & (G::RING - 1u)); };
        auto ring_drain = [&]() {
            if (ld_ready < ld_next) {   // chunks issued beyond what was read (look-ahead margin)
                wait_vm<0>();
                sync();
            }
            ld_next = 0;
            ld_ready = 0;
            partial_mask = 0;
        };
        // Make the bytes of the enumerating node's next ensemble (fpos, e items) readable:
        // one byte before it (word starts look back) and, for the text kind, a look-ahead
        // margin for the word-length node.  False only on an internal logic error.
        auto f_stage = [&](uint32_t fpos_, uint32_t fj_, uint32_t e) -> bool {
            if (!e) return true;
            uint32_t need_lo, need_hi;
            if constexpr (!BYTES) {
                need_lo = fpos_ * 4u;
                need_hi = (fpos_ + e) * 4u;
            } else {
                const uint32_t adr0 = TAG ? fpos_ : uni(SX[fj_]) + (fpos_ - uni(VT[fj_]));
                need_lo = adr0 > A0 ? adr0 - 1u : A0;
                need_hi = adr0 + e + 64u;
                if (need_hi > b1) need_hi = b1;
            }
            refill(need_lo);
            const uint32_t last_chunk = (need_hi - 1u - A0) / G::CHB;
            // one ensemble spans far less than NS-1 chunks, so refill has issued it
            if (ld_next <= last_chunk) return false;
            ready_upto(last_chunk);
            return true;
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
        // The enumerating node for one firing: items fpos + k*W + lane, k < V, of which the
        // first e are real.  Fetches each element under its parent's context and applies the
        // first stage.  keep[k], item[k], aux[k], reg[k] describe item k of this lane.
        auto f_fire = [&](uint32_t fpos_, uint32_t fj_, uint32_t jlo_, uint32_t e, uint32_t (&keep)[V],
                          uint32_t (&item)[V], uint32_t (&aux)[V], uint32_t (&reg)[V]) {
            uint32_t jr = jlo_;
#pragma unroll
            for (int k = 0; k < V; ++k) {
                keep[k] = 0;
                aux[k] = 0;
                const uint32_t i = (uint32_t)k * W + t;
                const uint32_t v = fpos_ + (i < e ? i : 0u);
                if constexpr (TAG) {
                    jr = (i < e) ? f_region(v, jr) : jr;
                    reg[k] = jr;
                } else {
                    reg[k] = fj_;
                }
            }
            if constexpr (!BYTES) {
                uint32_t addr[V], x[V];
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const uint32_t i = (uint32_t)k * W + t;
                    addr[k] = ring_off((fpos_ + (i < e ? i : 0u)) * 4u);
                }
                ring_read<V>(addr, x);
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const bool act = (uint32_t)k * W + t < e;
                    item[k] = x[k];
                    if constexpr (KIND == RS_MODFILTER) {
                        keep[k] = act && (mod_pow2 ? ((x[k] & (modm - 1u)) == modr) : (x[k] % modm == modr));
                    } else if constexpr (KIND == RS_HASH_EXPAND) {
                        const uint32_t h = fmix32(x[k] ^ salt_key(0));
                        keep[k] = act && (h & 1u);
                        aux[k] = (h >> 1) & 3u;
                    } else {
                        keep[k] = act && x[k] < CX[reg[k]];
                    }
                }
            } else {
                uint32_t ab[2 * V], bv[2 * V];
                bool in_line[V], at_start[V];
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const uint32_t i = (uint32_t)k * W + t;
                    const uint32_t v = fpos_ + i;
                    const uint32_t j = reg[k];
                    // signal: v is VT[j] plus the line-relative position; tag: v is the address
                    const uint32_t ls = SX[j];
                    const uint32_t adr = TAG ? v : ls + (v - VT[j]);
                    item[k] = adr;
                    in_line[k] = i < e && (!TAG || adr < ls + (VT[j + 1] - VT[j]));
                    at_start[k] = adr == ls;
                    ab[2 * k] = in_line[k] ? ring_off(adr) : ring_base;
                    ab[2 * k + 1] = (in_line[k] && !at_start[k]) ? ring_off(adr - 1u) : ring_base;
                }
                ring_read_u8<2 * V>(ab, bv);
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const uint32_t prev = at_start[k] ? 32u : bv[2 * k + 1];
                    keep[k] = in_line[k] && (bv[2 * k] != 32u) && (prev == 32u);
                }
            }
        };

        bool failed = false;
        // ---- ordered output stream: count this claim's outputs, then learn its base from the
        // claims before it (decoupled look-back over the stream's claims) before producing.
        uint32_t out_base_lo = 0, out_base_hi = 0;
        if (a.emit_outputs) {
            refill(A0);
            uint32_t fpos = vbeg, fj = 0, jlo = 0;
            bool fdone = TAG ? (vbeg >= vend) : (nb == 0);
            unsigned long long n_out = 0;
            while (!fdone) {
                const uint32_t e = TAG ? min(EW, vend - fpos) : min(EW, uni(VT[fj + 1]) - fpos);
                if (!f_stage(fpos, fj, e)) {
                    failed = true;
                    break;
                }
                uint32_t keep[V], item[V], aux[V], reg[V], nout[V], off[V], tot;
                f_fire(fpos, fj, jlo, e, keep, item, aux, reg);
#pragma unroll
                for (int k = 0; k < V; ++k) nout[k] = keep[k] ? (KIND == RS_HASH_EXPAND ? aux[k] : 1u) : 0u;
                ens_scan<W, V, true>(nout, off, tot, misc);
                n_out += tot;
                if constexpr (TAG) {
#pragma unroll
                    for (int k = 0; k < V; ++k)
                        if ((uint32_t)k * W + t == e - 1u) misc[M_JLAST] = reg[k];
                }
                fpos += e;
                sync();
                if constexpr (TAG) {
                    jlo = uni(misc[M_JLAST]);
                    fdone = (fpos == vend);
                } else {
                    if (fpos == uni(VT[fj + 1])) {
                        ++fj;
                        fdone = (fj == nb);
                    }
                }
            }
            ring_drain();
            // look-back: words are (epoch tag << 40) | (flag << 38) | value, flag 1 = this claim's
            // own count, flag 2 = inclusive prefix through this claim
            if (t == 0) {
                unsigned long long *lb = sd.lookback;
                const unsigned long long tagw = (unsigned long long)epoch_tag << 40;
                const unsigned long long mask38 = (1ull << 38) - 1ull;
                __hip_atomic_store(&lb[cidx], tagw | (1ull << 38) | (n_out & mask38), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                unsigned long long prefix = 0;
                for (uint32_t i = cidx; i-- > 0;) {
                    unsigned long long w;
                    for (;;) {
                        w = __hip_atomic_load(&lb[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if ((w >> 40) == (unsigned long long)epoch_tag && ((w >> 38) & 3ull)) break;
                        __builtin_amdgcn_s_sleep(2);
                    }
                    prefix += w & mask38;
                    if (((w >> 38) & 3ull) == 2ull) break;
                }
                __hip_atomic_store(&lb[cidx], tagw | (2ull << 38) | ((prefix + n_out) & mask38), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                misc[M_BASE_LO] = (uint32_t)prefix;
                misc[M_BASE_HI] = (uint32_t)(prefix >> 32);
            }
            sync();
            out_base_lo = uni(misc[M_BASE_LO]);
            out_base_hi = uni(misc[M_BASE_HI]);
        }
        uint32_t *const out_items = sd.out_items;
        unsigned long long out_rank = ((unsigned long long)out_base_hi << 32) | out_base_lo;

        refill(A0);

        // ---- node state (all uniform)
        uint32_t h1 = 0, t1 = 0, sh1 = 0, st1 = 0;
        uint32_t h2 = 0, t2 = 0, sh2 = 0, st2 = 0;
        // enumerating node: signal strategy walks region fj at position fpos;
        // tag strategy walks ensembles of EW consecutive positions from fpos.
        uint32_t fj = 0, fpos = vbeg, jlo = 0, ej = 0;
        bool fdone = TAG ? (vbeg >= vend) : (nb == 0);
        uint32_t a_items = 0;                 // items aggregated since the last signal (signal strategy)
        Acc acc;
        acc_reset(acc);
        uint32_t acc_tag = 0xFFFFFFFFu;       // tag strategy: region of this lane's running accumulator
        uint64_t st_fire[3] = {0, 0, 0}, st_items[3] = {0, 0, 0}, st_full[3] = {0, 0, 0}, st_sig[3] = {0, 0, 0};
        // every scheduler iteration fires a node; a claim needs at most a few firings per
        // element and per region, so this bound only trips on a scheduling error
        const unsigned long long iter_cap = 8ull * ((unsigned long long)(vend - vbeg) + nb) + 64ull;
        unsigned long long iters = 0;

        auto flush_tag = [&]() {
            if (acc.cnt) {
                atomicAdd(&s_cnt[acc_tag], acc.cnt);
                atomicAdd(&s_sum[acc_tag], acc.sum);
                atomicMin(&s_min[acc_tag], acc.mn);
                atomicMax(&s_max[acc_tag], acc.mx);
                acc_reset(acc);
            }
        };

        for (;;) {
            if (++iters > iter_cap) {
                failed = true;
                break;
            }
            // ---------------- A: the aggregating node (drains first)
            {
                uint32_t &h = HAS_E ? h2 : h1;
                uint32_t &sh = HAS_E ? sh2 : sh1;
                const uint32_t tq = HAS_E ? t2 : t1;
                const uint32_t stq = HAS_E ? st2 : st1;
                const uint32_t *qv = HAS_E ? q2v : q1v;
                const uint16_t *qt = HAS_E ? q2t : q1t;
                const uint32_t *sp = HAS_E ? sp2 : sp1;
                constexpr uint32_t D = HAS_E ? G::D2 : G::D1;
                const bool up_done = HAS_E ? (fdone && h1 == t1) : fdone;
                uint32_t e = 0;
                bool fire = false;
                if (!TAG && sh < stq) {
                    const uint32_t credit = uni(sp[sh & (G::SQ - 1u)]) - h;
                    e = credit < EW ? credit : EW;
                    fire = true;
                } else {
                    const uint32_t n = tq - h;
                    if (n >= EW) {
                        e = EW;
                        fire = true;
                    } else if (up_done && n > 0) {
                        e = n;
                        fire = true;
                    }
                }
                if (fire) {
                    if (e) {
#pragma unroll
                        for (int k = 0; k < V; ++k) {
                            const uint32_t i = (uint32_t)k * W + t;
                            if (i < e) {
                                const uint32_t pos = (h + i) & (D - 1u);
                                uint32_t y = qv[pos];
                                // the expansion's children arrive as pre-images x ^ K(j+1);
                                // finishing the hash here completes H(x, j+1)
                                if constexpr (KIND == RS_HASH_EXPAND) y = fmix32(y);
                                if (out_items) out_items[out_rank + i] = y;   // serial order
                                if constexpr (TAG) {
                                    const uint32_t tg = qt[pos];
                                    if (tg != acc_tag) {
                                        flush_tag();
                                        acc_tag = tg;
                                    }
                                }
                                acc_add(acc, y);
                            }
                        }
                        h += e;
                        a_items += e;
                        out_rank += e;
                        st_fire[2] += 1;
                        st_items[2] += e;
                        st_full[2] += (e == EW);
                    }
                    if constexpr (!TAG) {
                        // signal phase: consume every slot that no item precedes
                        while (sh < stq && uni(sp[sh & (G::SQ - 1u)]) == h) {
                            const uint32_t j = uni(qv[h & (D - 1u)]);
                            if (a_items) {
                                const Acc r = wg_reduce<W>(acc, misc);
                                if (t == 0) {
                                    s_cnt[j] = r.cnt;
                                    s_sum[j] = r.sum;
                                    s_min[j] = r.mn;
                                    s_max[j] = r.mx;
                                }
                                acc_reset(acc);
                                a_items = 0;
                            }
                            ++h;
                            ++sh;
                            st_sig[2] += 1;
                        }
                    }
                    sync();
                    continue;
                }
            }
            // ---------------- E: the second node
            if constexpr (HAS_E) {
                uint32_t e = 0;
                bool fire = false;
                const uint32_t space = G::D2 - (t2 - h2) - (TAG ? 0u : 1u);
                const uint32_t cap = space / KE;
                if (!TAG && sh1 < st1) {
                    const uint32_t credit = uni(sp1[sh1 & (G::SQ - 1u)]) - h1;
                    e = min(min(credit, EW), cap);
                    fire = (credit == 0) ? (space >= 1u && st2 - sh2 < G::SQ) : (e > 0);
                } else {
                    const uint32_t n = t1 - h1;
                    if (n >= EW || (fdone && n > 0)) {
                        e = min(min(n, EW), cap);
                        fire = e > 0;
                    }
                }
                if (fire) {
                    if (e) {
                        uint32_t nout[V], x[V], tg[V], off[V], tot;
#pragma unroll
                        for (int k = 0; k < V; ++k) {
                            const uint32_t i = (uint32_t)k * W + t;
                            nout[k] = 0;
                            x[k] = 0;
                            tg[k] = 0;
                            if (i < e) {
                                const uint32_t pos = (h1 + i) & (G::D1 - 1u);
                                x[k] = q1v[pos];
                                if constexpr (TAG) tg[k] = q1t[pos];
                                if constexpr (KIND == RS_HASH_EXPAND) {
                                    nout[k] = q1a[pos];
                                } else {
                                    // word length: run of non-space bytes from the start, within the line,
                                    // read four bytes at a time from the ring (global memory outside it)
                                    const uint32_t j = TAG ? tg[k] : ej;
                                    const uint32_t le = SX[j] + (VT[j + 1] - VT[j]);
                                    const uint32_t wlo = A0 + (ld_next > G::NS ? ld_next - G::NS : 0u) * G::CHB;
                                    const uint32_t whi = A0 + ld_ready * G::CHB;
                                    uint32_t p = x[k];
                                    while (p < le) {
                                        const uint32_t q = p & ~3u;
                                        uint32_t word = 0;
                                        if (q >= wlo && q + 8u <= whi) {
                                            uint32_t w0, w1;
                                            ring_u32x2(ring_off(q), ring_off(q + 4u), w0, w1);
                                            word = __builtin_amdgcn_alignbyte(w1, w0, p & 3u);
                                        } else {
                                            for (uint32_t b = 0; b < 4u && p + b < le; ++b)
                                                word |= (uint32_t)elems[p + b] << (8u * b);
                                        }
                                        // first space among the four bytes: zero byte of word ^ "    "
                                        const uint32_t z = word ^ 0x20202020u;
                                        const uint32_t zm = (z - 0x01010101u) & ~z & 0x80808080u;
                                        uint32_t step = zm ? ((uint32_t)__builtin_ctz(zm) >> 3) : 4u;
                                        if (le - p < step) step = le - p;
                                        p += step;
                                        if (step < 4u) break;
                                    }
                                    x[k] = p - x[k];
                                    nout[k] = 1;
                                }
                            }
                        }
                        ens_scan<W, V, KE == 3>(nout, off, tot, misc);
#pragma unroll
                        for (int k = 0; k < V; ++k) {
                            const uint32_t base = t2 + off[k];
                            if constexpr (KIND == RS_HASH_EXPAND) {
                                // child j of x leaves as its pre-image x ^ K(j+1)
                                if (nout[k] > 0) q2v[base & (G::D2 - 1u)] = x[k] ^ salt_key(1);
                                if (nout[k] > 1) q2v[(base + 1u) & (G::D2 - 1u)] = x[k] ^ salt_key(2);
                                if (nout[k] > 2) q2v[(base + 2u) & (G::D2 - 1u)] = x[k] ^ salt_key(3);
                                if constexpr (TAG) {
                                    if (nout[k] > 0) q2t[base & (G::D2 - 1u)] = (uint16_t)tg[k];
                                    if (nout[k] > 1) q2t[(base + 1u) & (G::D2 - 1u)] = (uint16_t)tg[k];
                                    if (nout[k] > 2) q2t[(base + 2u) & (G::D2 - 1u)] = (uint16_t)tg[k];
                                }
                            } else {
                                if (nout[k]) {
                                    q2v[base & (G::D2 - 1u)] = x[k];
                                    if constexpr (TAG) q2t[base & (G::D2 - 1u)] = (uint16_t)tg[k];
                                }
                            }
                        }
                        h1 += e;
                        t2 += tot;
                        st_fire[1] += 1;
                        st_items[1] += e;
                        st_full[1] += (e == EW);
                    }
                    if constexpr (!TAG) {
                        while (sh1 < st1 && uni(sp1[sh1 & (G::SQ - 1u)]) == h1 && G::D2 - (t2 - h2) >= 1u &&
                               st2 - sh2 < G::SQ) {
                            const uint32_t j = uni(q1v[h1 & (G::D1 - 1u)]);
                            if (t == 0) {
                                q2v[t2 & (G::D2 - 1u)] = j;
                                sp2[st2 & (G::SQ - 1u)] = t2;
                            }
                            ++t2;
                            ++st2;
                            ++h1;
                            ++sh1;
                            ++ej;
                            st_sig[1] += 1;
                        }
                    }
                    sync();
                    continue;
                }
            }
            // ---------------- F: the enumerating node
            if (!fdone) {
                uint32_t e, j_sig = 0;
                bool ends_region = false;
                if constexpr (TAG) {
                    e = min(EW, vend - fpos);
                } else {
                    const uint32_t rend = uni(VT[fj + 1]);
                    e = min(EW, rend - fpos);
                    ends_region = (fpos + e == rend);
                    j_sig = fj;
                }
                const uint32_t space1 = G::D1 - (t1 - h1);
                const bool sig_ok = TAG || !ends_region || (st1 - sh1 < G::SQ);
                if (space1 >= e + (ends_region ? 1u : 0u) && sig_ok) {
                    if (!f_stage(fpos, fj, e)) {
                        failed = true;
                        break;
                    }
                    uint32_t keep[V], item[V], aux[V], reg[V], off[V], tot;
                    f_fire(fpos, fj, jlo, e, keep, item, aux, reg);
                    ens_scan<W, V, false>(keep, off, tot, misc);
#pragma unroll
                    for (int k = 0; k < V; ++k) {
                        if (keep[k]) {
                            const uint32_t pos = (t1 + off[k]) & (G::D1 - 1u);
                            q1v[pos] = item[k];
                            if constexpr (KIND == RS_HASH_EXPAND) q1a[pos] = (uint8_t)aux[k];
                            if constexpr (TAG) q1t[pos] = (uint16_t)reg[k];
                        }
                        if constexpr (TAG) {
                            if ((uint32_t)k * W + t == e - 1u) misc[M_JLAST] = reg[k];
                        }
                    }
                    t1 += tot;
                    fpos += e;
                    if (e) {
                        st_fire[0] += 1;
                        st_items[0] += e;
                        st_full[0] += (e == EW);
                    }
                    if constexpr (!TAG) {
                        if (ends_region) {
                            if (t == 0) {
                                q1v[t1 & (G::D1 - 1u)] = j_sig;
                                sp1[st1 & (G::SQ - 1u)] = t1;
                            }
                            ++t1;
                            ++st1;
                            ++fj;
                            st_sig[0] += 1;
                            fdone = (fj == nb);
                        }
                    }
                    sync();
                    if constexpr (TAG) {
                        if (e) jlo = uni(misc[M_JLAST]);
                        fdone = (fpos == vend);
                    }
                    continue;
                }
            }
            // nothing fireable
            if (fdone && h1 == t1 && h2 == t2) break;
            failed = true;   // cannot happen: some node is always fireable (Lemma 2)
            break;
        }

        if constexpr (TAG) {
            flush_tag();
            sync();
        }
        ring_drain();
        if (failed && t == 0) atomicOr(&a.ctl[CTL_ERROR], 1u);

        // ---- end(): one record per parent, written once
        for (uint32_t i = t; i < nb; i += W) {
            const uint32_t p = p0 + i;
            if (a.agg_fields & RS_COUNT) sd.agg_count[p] = s_cnt[i];
            if (a.agg_fields & RS_SUM) sd.agg_sum[p] = s_sum[i];
            if (a.agg_fields & RS_MIN) sd.agg_min[p] = s_min[i];
            if (a.agg_fields & RS_MAX) sd.agg_max[p] = s_max[i];
        }
        if (a.collect_stats && t == 0) {
            for (int k = 0; k < 3; ++k) {
                atomicAdd(&sd.stats[ST_FIRINGS + k], (unsigned long long)st_fire[k]);
                atomicAdd(&sd.stats[ST_ITEMS + k], (unsigned long long)st_items[k]);
                atomicAdd(&sd.stats[ST_FULL + k], (unsigned long long)st_full[k]);
                atomicAdd(&sd.stats[ST_SIGNALS + k], (unsigned long long)st_sig[k]);
            }
        }
        if (t == 0) misc[M_NEXT] = g_next;
        sync();
        g = g1;
        g1 = uni(misc[M_NEXT]);
        cur = nxt;
    }

    // last workgroup out returns the control block to zero for the next launch
    if (t == 0) {
        __threadfence();
        const uint32_t d = atomicAdd(&a.ctl[CTL_DONE], 1u);
        if (d == gridDim.x - 1u) {
            atomicExch(&a.ctl[CTL_CLAIM], 0u);
            atomicExch(&a.ctl[CTL_DONE], 0u);
            atomicAdd(&a.ctl[CTL_EPOCH], 1u);
        }
    }
}

// ---------------------------------------------------------------- launch table

using KernelFn = void (*)(LaunchArgs);

// Ensemble width w = W * V: W lanes per workgroup, V items per lane per firing.  Every width
// runs on single-wave processors: a wave's lanes share one scheduler with no barrier.
template <int KIND, int STRAT>
static KernelFn pick_width(uint32_t w) {
    switch (w) {
        case 64: return rs_pipeline<KIND, STRAT, 64, 1>;
        case 128: return rs_pipeline<KIND, STRAT, 64, 2>;
        case 256: return rs_pipeline<KIND, STRAT, 64, 4>;
        case 512: return rs_pipeline<KIND, STRAT, 64, 8>;
        case 1024: return rs_pipeline<KIND, STRAT, 64, 16>;
        default: return nullptr;
    }
}

template <int KIND>
static KernelFn pick_strategy(uint32_t s, uint32_t w) {
    return s == RS_TAG ? pick_width<KIND, RS_TAG>(w) : s == RS_SIGNAL ? pick_width<KIND, RS_SIGNAL>(w) : nullptr;
}

static KernelFn pick(uint32_t kind, uint32_t s, uint32_t w) {
    switch (kind) {
        case RS_MODFILTER: return pick_strategy<RS_MODFILTER>(s, w);
        case RS_HASH_EXPAND: return pick_strategy<RS_HASH_EXPAND>(s, w);
        case RS_TEXT_WORDS: return pick_strategy<RS_TEXT_WORDS>(s, w);
        case RS_GRAPH_THRESH: return pick_strategy<RS_GRAPH_THRESH>(s, w);
        default: return nullptr;
    }
}

uint32_t lanes_of(uint32_t ensemble_width) { return ensemble_width ? 64u : 0u; }

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

bool kernel_supported(uint32_t kind, uint32_t strategy, uint32_t width) {
    return pick(kind, strategy, width) != nullptr;
}

int launch_pipeline(uint32_t kind, uint32_t strategy, uint32_t width, const LaunchArgs &a, uint32_t grid,
                    void *stream) {
    KernelFn k = pick(kind, strategy, width);
    if (!k) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(grid), dim3(lanes_of(width)), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int blocks_per_cu(uint32_t kind, uint32_t strategy, uint32_t width) {
    KernelFn k = pick(kind, strategy, width);
    if (!k) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, (int)lanes_of(width), 0) != hipSuccess) return 0;
    return n;
}

}  // namespace rs
