// gfx950 kernels of the region-stateful streaming pipeline.
//
// One workgroup of W lanes is one SIMD processor in the sense of §2.2: it runs a
// whole pipeline instance (enumerating node F, optional second node E, aggregating
// node A) with a non-preemptive scheduler, and it competes with every other
// workgroup for parent batches ("claims") through a device atomic on a common
// counter, returning only when every claim of every stream in the launch is done.
// A firing of a node consumes an ensemble of at most W items, one per lane.
//
// Nodes are joined by fixed-size LDS queues.  Data-dependent output counts are
// compacted with wave64 ballot/mbcnt ranks plus an LDS prefix over the waves.
// Region boundaries travel either
//   - as signals (RS_SIGNAL): an end-of-region slot sits in the queue at its exact
//     stream position; the items between two slots are that signal's credit (the
//     in-band form of the credit protocol of §3.1), a consumer's ensemble never
//     extends past the next slot (the SIMD rule of §3.3), and a node consumes a
//     slot only when no item precedes it, running end() for that region; or
//   - as tags (RS_TAG): every queued item carries its region index, ensembles mix
//     regions freely, and the aggregating node reduces by tag (§5).
// Aggregates are exact integer reductions kept in LDS slots per claim and written
// once per parent; a claim always holds whole regions, so no aggregate is ever
// shared between workgroups.
//
// Elements reach the enumerating node through an LDS ring filled by direct
// global->LDS loads (global_load_lds_dwordx4), NS chunks deep, independent of
// where ensembles or regions begin.  The compiler does not track which chunk a
// read touches, so the ring is read with inline-asm ds_read and completion is
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
__device__ __forceinline__ uint32_t salt_key(uint32_t s) { return 0x9E3779B9u * (s + 1u); }

// ---------------------------------------------------------------- wave / workgroup helpers

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Workgroup barrier that waits for this wave's LDS operations only (not for
// outstanding global->LDS chunk loads, whose completion is waited for explicitly).
__device__ __forceinline__ void bar() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

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
__device__ __forceinline__ uint32_t ring_u8(uint32_t addr) {
    uint32_t v;
    asm volatile("ds_read_u8 %0, %1\n\ts_waitcnt lgkmcnt(0)" : "=v"(v) : "v"(addr) : "memory");
    return v;
}
__device__ __forceinline__ void ring_w8(uint32_t addr, uint32_t v) {
    asm volatile("ds_write_b8 %0, %1\n\ts_waitcnt lgkmcnt(0)" : : "v"(addr), "v"(v) : "memory");
}

// Exclusive prefix of small per-lane counts n in [0, 3] over the workgroup.
template <int W>
__device__ __forceinline__ uint32_t wg_scan3(uint32_t n, uint32_t *scr, uint32_t &total) {
    const uint64_t b0 = __ballot(n & 1u);
    const uint64_t b1 = __ballot((n >> 1) & 1u);
    const uint32_t within = rank_below(b0) + 2u * rank_below(b1);
    const uint32_t wsum = (uint32_t)__popcll(b0) + 2u * (uint32_t)__popcll(b1);
    if constexpr (W == 64) {
        total = uni(wsum);
        return within;
    } else {
        const uint32_t wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63u) == 0) scr[wv] = wsum;
        bar();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (uint32_t i = 0; i < (uint32_t)W / 64u; ++i) {
            const uint32_t s = scr[i];
            before += (i < wv) ? s : 0u;
            all += s;
        }
        total = uni(all);
        return before + within;
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
            scr[16 + wv] = a.cnt;
            scr[32 + 2 * wv] = (uint32_t)a.sum;
            scr[33 + 2 * wv] = (uint32_t)(a.sum >> 32);
            scr[64 + wv] = a.mn;
            scr[80 + wv] = a.mx;
        }
        bar();
        Acc r;
        acc_reset(r);
#pragma unroll
        for (uint32_t i = 0; i < NW; ++i) {
            r.cnt += scr[16 + i];
            r.sum += (unsigned long long)scr[32 + 2 * i] | ((unsigned long long)scr[33 + 2 * i] << 32);
            r.mn = r.mn < scr[64 + i] ? r.mn : scr[64 + i];
            r.mx = r.mx > scr[80 + i] ? r.mx : scr[80 + i];
        }
        return r;
    }
}

// ---------------------------------------------------------------- geometry

template <int W>
struct Geo {
    static constexpr uint32_t BMAX = W;          // parents in one claim, at most
    static constexpr uint32_t D1 = 2 * W;        // slots of the queue in front of the second node
    static constexpr uint32_t D2 = 4 * W;        // slots of the queue in front of the third node
    static constexpr uint32_t CHB = 16 * W;      // bytes of one ring chunk: one 16-byte load per lane
    static constexpr uint32_t NS = 4;            // chunks in the element ring
    static constexpr uint32_t RING = NS * CHB;
};

enum Misc : uint32_t { M_NEXT = 100, M_JLAST = 101, M_PARTIAL = 102 };

// ---------------------------------------------------------------- the pipeline kernel

template <int KIND, int STRAT, int W>
__global__ void __launch_bounds__(W) rs_pipeline(LaunchArgs a) {
    using G = Geo<W>;
    constexpr bool TAG = (STRAT == RS_TAG);
    constexpr bool HAS_E = (KIND == RS_HASH_EXPAND || KIND == RS_TEXT_WORDS);
    constexpr bool BYTES = (KIND == RS_TEXT_WORDS);
    constexpr bool CTXP = (KIND == RS_GRAPH_THRESH);
    constexpr uint32_t EB = BYTES ? 1u : 4u;          // element bytes
    constexpr uint32_t KE = (KIND == RS_HASH_EXPAND) ? 3u : 1u;   // outputs per input of E

    __shared__ __attribute__((aligned(16))) uint8_t ring[G::RING];
    __shared__ uint32_t V[G::BMAX + 1];
    __shared__ uint32_t SX[BYTES ? G::BMAX : 1];
    __shared__ uint32_t CX[CTXP ? G::BMAX : 1];
    __shared__ uint32_t s_cnt[G::BMAX];
    __shared__ unsigned long long s_sum[G::BMAX];
    __shared__ uint32_t s_min[G::BMAX];
    __shared__ uint32_t s_max[G::BMAX];
    __shared__ uint32_t q1v[G::D1];
    __shared__ uint32_t q1a[KIND == RS_HASH_EXPAND ? G::D1 : 1];
    __shared__ uint32_t q1t[TAG ? G::D1 : 1];
    __shared__ uint32_t sp1[TAG ? 1 : G::D1];
    __shared__ uint32_t q2v[HAS_E ? G::D2 : 1];
    __shared__ uint32_t q2t[(HAS_E && TAG) ? G::D2 : 1];
    __shared__ uint32_t sp2[(HAS_E && !TAG) ? G::D2 : 1];
    __shared__ uint32_t misc[128];

    const uint32_t t = threadIdx.x;
    const uint32_t wv = t >> 6;
    const uint32_t ring_base = lds_addr(ring);

    // stage parameters
    const uint32_t modm = a.param[0] ? a.param[0] : 4u;
    const uint32_t modr = a.param[1];
    const bool mod_pow2 = (modm & (modm - 1u)) == 0u;

    if (t == 0) misc[M_NEXT] = atomicAdd(&a.ctl[CTL_CLAIM], 1u);
    bar();
    uint32_t g = uni(misc[M_NEXT]);

    while (g < a.total_claims) {
        uint32_t g_next = 0;
        if (t == 0) g_next = atomicAdd(&a.ctl[CTL_CLAIM], 1u);   // overlaps with this claim

        // stream of this claim: the last with claim_begin <= g
        uint32_t lo = 0, hi = a.n_streams;
        while (hi - lo > 1u) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.streams[mid].claim_begin <= g) lo = mid; else hi = mid;
        }
        const StreamDev &sd = a.streams[lo];
        const uint8_t *elems = (const uint8_t *)sd.elements;
        const uint32_t B = sd.parents_per_claim;
        const uint32_t p0 = (g - sd.claim_begin) * B;
        const uint32_t nb = uni(min(B, sd.n_parents - p0));
        const uint32_t nbytes_total = sd.n_elements * EB;

        // ---- region table of the claim (enumeration: findCount per parent)
        uint32_t vbeg, vend;
        if constexpr (!BYTES) {
            for (uint32_t i = t; i <= nb; i += W) V[i] = sd.offsets[p0 + i];
            if constexpr (CTXP)
                for (uint32_t i = t; i < nb; i += W) CX[i] = sd.pparam[p0 + i];
            bar();
            vbeg = uni(V[0]);
            vend = uni(V[nb]);
        } else {
            uint32_t carry = 0;
            for (uint32_t i0 = 0; i0 < nb; i0 += W) {
                const uint32_t i = i0 + t;
                uint32_t len = 0;
                if (i < nb) {
                    SX[i] = sd.offsets[p0 + i];
                    len = sd.lengths[p0 + i];
                }
                uint32_t tot;
                const uint32_t ex = wg_scan_u32<W>(len, misc, tot);
                if (i < nb) V[i] = carry + ex;
                carry += tot;
                bar();
            }
            if (t == 0) V[nb] = carry;
            bar();
            vbeg = 0;
            vend = carry;
        }
        for (uint32_t i = t; i < nb; i += W) {
            s_cnt[i] = 0;
            s_sum[i] = 0ull;
            s_min[i] = 0xFFFFFFFFu;
            s_max[i] = 0;
        }

        // ---- element ring: the claim's byte range, chunked from a 16-byte aligned base
        uint32_t b0, b1;
        if constexpr (!BYTES) {
            b0 = vbeg * 4u;
            b1 = vend * 4u;
        } else {
            b0 = nb ? uni(SX[0]) : 0u;
            b1 = nb ? uni(SX[nb - 1] + (V[nb] - V[nb - 1])) : 0u;
        }
        if constexpr (BYTES && TAG) {   // lines are enumerated over the claim's address range
            vbeg = b0;
            vend = b1;
        }
        const uint32_t A0 = b0 & ~15u;
        const uint32_t nch = (b1 > b0) ? (b1 - A0 + G::CHB - 1u) / G::CHB : 0u;
        uint32_t ld_next = 0, ld_ready = 0;
        uint32_t partial_mask = 0;   // per lane: chunk-parity bits of a pending partial tail block

        auto issue = [&]() {
            const uint32_t c = ld_next;
            const uint32_t blk = A0 + c * G::CHB + t * 16u;
            const bool full = blk + 16u <= nbytes_total;
            const uint8_t *src = full ? elems + blk : (const uint8_t *)a.dummy;
            if (!full && blk < nbytes_total) partial_mask |= 1u << (c % G::NS);
            __builtin_amdgcn_global_load_lds((glb_void_t *)src,
                                             (lds_void_t *)(ring + (c % G::NS) * G::CHB + wv * 1024u),
                                             16, 0, 0);
            ld_next = c + 1u;
        };
        // make chunks [0, k] readable
        auto ready_upto = [&](uint32_t k) {
            while (ld_ready <= k) {
                const uint32_t after = ld_next - 1u - ld_ready;
                wait_vm_n(after);
                if (partial_mask & (1u << (ld_ready % G::NS))) {
                    partial_mask &= ~(1u << (ld_ready % G::NS));
                    const uint32_t blk = A0 + ld_ready * G::CHB + t * 16u;
                    const uint32_t dst = ring_base + (ld_ready % G::NS) * G::CHB + t * 16u;
                    for (uint32_t k2 = 0; blk + k2 < nbytes_total; ++k2) ring_w8(dst + k2, elems[blk + k2]);
                }
                bar();
                ++ld_ready;
            }
        };
        // issue every chunk whose ring slot is free: chunk ld_next reuses the slot of
        // chunk ld_next - NS, which must end at or before need_from
        auto refill = [&](uint32_t need_from) {
            while (ld_next < nch &&
                   (ld_next < G::NS || A0 + (ld_next - G::NS + 1u) * G::CHB <= need_from))
                issue();
        };
        auto ring_off = [&](uint32_t addr) -> uint32_t { return ring_base + ((addr - A0) & (G::RING - 1u)); };

        refill(A0);
        bar();   // slots initialised, region table visible

        // ---- node state (all uniform)
        uint32_t h1 = 0, t1 = 0, sh1 = 0, st1 = 0;
        uint32_t h2 = 0, t2 = 0, sh2 = 0, st2 = 0;
        // enumerating node: signal strategy walks region j at position fpos;
        // tag strategy walks ensembles of W consecutive elements from fpos.
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
        bool failed = false;

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
            if (++iters > iter_cap) { failed = true; break; }
            // ---------------- A: the aggregating node (drains first)
            {
                uint32_t &h = HAS_E ? h2 : h1;
                uint32_t &tq = HAS_E ? t2 : t1;
                uint32_t &sh = HAS_E ? sh2 : sh1;
                const uint32_t &stq = HAS_E ? st2 : st1;
                const uint32_t *qv = HAS_E ? q2v : q1v;
                const uint32_t *qt = HAS_E ? q2t : q1t;
                const uint32_t *sp = HAS_E ? sp2 : sp1;
                constexpr uint32_t D = HAS_E ? G::D2 : G::D1;
                const bool up_done = HAS_E ? (fdone && h1 == t1) : fdone;
                uint32_t e = 0;
                bool fire = false, sig_next = false;
                if (!TAG && sh < stq) {
                    const uint32_t credit = uni(sp[sh & (D - 1u)]) - h;
                    e = credit < (uint32_t)W ? credit : (uint32_t)W;
                    fire = true;
                    sig_next = true;
                } else {
                    const uint32_t n = tq - h;
                    if (n >= (uint32_t)W) { e = W; fire = true; }
                    else if (up_done && n > 0) { e = n; fire = true; }
                }
                if (fire) {
                    if (e) {
                        if (t < e) {
                            const uint32_t pos = (h + t) & (D - 1u);
                            const uint32_t y = qv[pos];
                            if constexpr (TAG) {
                                const uint32_t tg = qt[pos];
                                if (tg != acc_tag) {
                                    flush_tag();
                                    acc_tag = tg;
                                }
                            }
                            acc_add(acc, y);
                        }
                        h += e;
                        a_items += e;
                        st_fire[2] += 1;
                        st_items[2] += e;
                        st_full[2] += (e == (uint32_t)W);
                    }
                    if constexpr (!TAG) {
                        // signal phase: consume every slot that no item precedes
                        while (sh < stq && uni(sp[sh & (D - 1u)]) == h) {
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
                    (void)sig_next;
                    bar();
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
                    const uint32_t credit = uni(sp1[sh1 & (G::D1 - 1u)]) - h1;
                    e = min(min(credit, (uint32_t)W), cap);
                    fire = (credit == 0) ? (space >= 1u) : (e > 0);
                } else {
                    const uint32_t n = t1 - h1;
                    if (n >= (uint32_t)W || (fdone && n > 0)) {
                        e = min(min(n, (uint32_t)W), cap);
                        fire = e > 0;
                    }
                }
                if (fire) {
                    if (e) {
                        uint32_t nout = 0, y0 = 0, y1 = 0, y2 = 0, tg = 0;
                        if (t < e) {
                            const uint32_t pos = (h1 + t) & (G::D1 - 1u);
                            const uint32_t x = q1v[pos];
                            if constexpr (TAG) tg = q1t[pos];
                            if constexpr (KIND == RS_HASH_EXPAND) {
                                nout = q1a[pos];
                                y0 = fmix32(x ^ salt_key(1));
                                y1 = fmix32(x ^ salt_key(2));
                                y2 = fmix32(x ^ salt_key(3));
                            } else {   // word length: run of non-space bytes from the start, within the line
                                const uint32_t j = TAG ? tg : ej;
                                const uint32_t le = SX[j] + (V[j + 1] - V[j]);
                                const uint32_t wlo = A0 + (ld_next > G::NS ? ld_next - G::NS : 0u) * G::CHB;
                                const uint32_t whi = A0 + ld_ready * G::CHB;
                                uint32_t p = x;
                                while (p < le) {
                                    const uint32_t b = (p >= wlo && p < whi) ? ring_u8(ring_off(p)) : (uint32_t)elems[p];
                                    if (b == 32u) break;
                                    ++p;
                                }
                                y0 = p - x;
                                nout = 1;
                            }
                        }
                        uint32_t tot;
                        const uint32_t off = wg_scan3<W>(nout, misc, tot);
                        if (t < e) {
                            const uint32_t base = t2 + off;
                            if (nout > 0) { q2v[base & (G::D2 - 1u)] = y0; if constexpr (TAG) q2t[base & (G::D2 - 1u)] = tg; }
                            if (nout > 1) { q2v[(base + 1u) & (G::D2 - 1u)] = y1; if constexpr (TAG) q2t[(base + 1u) & (G::D2 - 1u)] = tg; }
                            if (nout > 2) { q2v[(base + 2u) & (G::D2 - 1u)] = y2; if constexpr (TAG) q2t[(base + 2u) & (G::D2 - 1u)] = tg; }
                        }
                        h1 += e;
                        t2 += tot;
                        st_fire[1] += 1;
                        st_items[1] += e;
                        st_full[1] += (e == (uint32_t)W);
                    }
                    if constexpr (!TAG) {
                        while (sh1 < st1 && uni(sp1[sh1 & (G::D1 - 1u)]) == h1 && G::D2 - (t2 - h2) >= 1u) {
                            const uint32_t j = uni(q1v[h1 & (G::D1 - 1u)]);
                            if (t == 0) {
                                q2v[t2 & (G::D2 - 1u)] = j;
                                sp2[st2 & (G::D2 - 1u)] = t2;
                            }
                            ++t2;
                            ++st2;
                            ++h1;
                            ++sh1;
                            ++ej;
                            st_sig[1] += 1;
                        }
                    }
                    bar();
                    continue;
                }
            }
            // ---------------- F: the enumerating node
            if (!fdone) {
                uint32_t e, j_sig = 0;
                bool ends_region = false;
                if constexpr (TAG) {
                    e = min((uint32_t)W, vend - fpos);
                } else {
                    const uint32_t rend = uni(V[fj + 1]);
                    e = min((uint32_t)W, rend - fpos);
                    ends_region = (fpos + e == rend);
                    j_sig = fj;
                }
                const uint32_t space1 = G::D1 - (t1 - h1);
                if (space1 >= e + (ends_region ? 1u : 0u)) {
                    // bytes this ensemble reads (plus one byte before it and a look-ahead
                    // margin for the word-length node under the text kind)
                    uint32_t need_lo, need_hi;
                    if constexpr (!BYTES) {
                        need_lo = fpos * 4u;
                        need_hi = (fpos + e) * 4u;
                    } else {
                        const uint32_t adr0 = TAG ? fpos : uni(SX[fj]) + (fpos - uni(V[fj]));
                        need_lo = adr0 > A0 ? adr0 - 1u : A0;
                        need_hi = adr0 + e + 64u;
                        if (need_hi > b1) need_hi = b1;
                    }
                    if (e) {
                        refill(need_lo);
                        const uint32_t last_chunk = (need_hi - 1u - A0) / G::CHB;
                        // the span of one ensemble is far below (NS-1) chunks, so refill has
                        // always issued it; anything else is a logic error
                        if (ld_next <= last_chunk) { failed = true; break; }
                        ready_upto(last_chunk);
                    }
                    uint32_t keep = 0, item = 0, aux = 0, tg = 0;
                    if (t < e) {
                        const uint32_t v = fpos + t;
                        uint32_t j;
                        if constexpr (TAG) {
                            // largest j with start(j) <= v: element index (CSR) or byte address (lines)
                            const uint32_t *key = BYTES ? SX : V;
                            uint32_t l2 = jlo, h2s = nb;
                            while (h2s - l2 > 1u) {
                                const uint32_t m = (l2 + h2s) >> 1;
                                if (key[m] <= v) l2 = m; else h2s = m;
                            }
                            j = l2;
                            tg = j;
                        } else {
                            j = fj;
                        }
                        if constexpr (KIND == RS_MODFILTER) {
                            const uint32_t x = ring_u32(ring_off(v * 4u));
                            keep = mod_pow2 ? ((x & (modm - 1u)) == modr) : (x % modm == modr);
                            item = x;
                        } else if constexpr (KIND == RS_HASH_EXPAND) {
                            const uint32_t x = ring_u32(ring_off(v * 4u));
                            const uint32_t h = fmix32(x ^ salt_key(0));
                            keep = h & 1u;
                            item = x;
                            aux = (h >> 1) & 3u;
                        } else if constexpr (KIND == RS_GRAPH_THRESH) {
                            const uint32_t x = ring_u32(ring_off(v * 4u));
                            keep = x < CX[j];
                            item = x;
                        } else {
                            // signal: v is the line-relative position plus V[j]; tag: v is the address
                            const uint32_t ls = SX[j];
                            const uint32_t adr = TAG ? v : ls + (v - V[j]);
                            const bool in_line = !TAG || adr < ls + (V[j + 1] - V[j]);
                            if (in_line) {
                                const uint32_t b = ring_u8(ring_off(adr));
                                const uint32_t prev = (adr == ls) ? 32u : ring_u8(ring_off(adr - 1u));
                                keep = (b != 32u) && (prev == 32u);
                            }
                            item = adr;
                        }
                    }
                    uint32_t tot;
                    const uint32_t off = wg_scan3<W>(keep, misc, tot);
                    if (keep) {
                        const uint32_t pos = (t1 + off) & (G::D1 - 1u);
                        q1v[pos] = item;
                        if constexpr (KIND == RS_HASH_EXPAND) q1a[pos] = aux;
                        if constexpr (TAG) q1t[pos] = tg;
                    }
                    if constexpr (TAG) {
                        if (t == e - 1u) misc[M_JLAST] = tg;
                    }
                    t1 += tot;
                    fpos += e;
                    if (e) {
                        st_fire[0] += 1;
                        st_items[0] += e;
                        st_full[0] += (e == (uint32_t)W);
                    }
                    if constexpr (!TAG) {
                        if (ends_region) {
                            if (t == 0) {
                                q1v[t1 & (G::D1 - 1u)] = j_sig;
                                sp1[st1 & (G::D1 - 1u)] = t1;
                            }
                            ++t1;
                            ++st1;
                            ++fj;
                            st_sig[0] += 1;
                            fdone = (fj == nb);
                        }
                    }
                    bar();
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
            bar();
        }
        if (ld_ready < ld_next) {   // chunks issued beyond what was read (look-ahead margin)
            wait_vm<0>();
            bar();
        }
        if (failed && t == 0) atomicOr(&a.ctl[CTL_ERROR], 1u);

        // ---- end(): one record per parent, written once
        for (uint32_t i = t; i < nb; i += W) {
            const uint32_t p = p0 + i;
            if (a.agg_fields & RS_COUNT) sd.agg_count[p] = s_cnt[i];
            if (a.agg_fields & RS_SUM) sd.agg_sum[p] = s_sum[i];
            if (a.agg_fields & RS_MIN) sd.agg_min[p] = s_min[i];
            if (a.agg_fields & RS_MAX) sd.agg_max[p] = s_max[i];
        }
        if (a.collect_stats && t == 0 && sd.stats) {
            for (int k = 0; k < 3; ++k) {
                atomicAdd(&sd.stats[ST_FIRINGS + k], (unsigned long long)st_fire[k]);
                atomicAdd(&sd.stats[ST_ITEMS + k], (unsigned long long)st_items[k]);
                atomicAdd(&sd.stats[ST_FULL + k], (unsigned long long)st_full[k]);
                atomicAdd(&sd.stats[ST_SIGNALS + k], (unsigned long long)st_sig[k]);
            }
        }
        if (t == 0) misc[M_NEXT] = g_next;
        bar();
        g = uni(misc[M_NEXT]);
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

}  // namespace rs

// ---------------------------------------------------------------- launch table

namespace rs {

using KernelFn = void (*)(LaunchArgs);

template <int KIND, int STRAT>
static KernelFn pick_width(uint32_t w) {
    switch (w) {
        case 64: return rs_pipeline<KIND, STRAT, 64>;
        case 128: return rs_pipeline<KIND, STRAT, 128>;
        case 256: return rs_pipeline<KIND, STRAT, 256>;
        case 512: return rs_pipeline<KIND, STRAT, 512>;
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

bool kernel_supported(uint32_t kind, uint32_t strategy, uint32_t width) {
    return pick(kind, strategy, width) != nullptr;
}

int launch_pipeline(uint32_t kind, uint32_t strategy, uint32_t width, const LaunchArgs &a,
                    uint32_t grid, void *stream) {
    KernelFn k = pick(kind, strategy, width);
    if (!k) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(grid), dim3(width), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
}

int blocks_per_cu(uint32_t kind, uint32_t strategy, uint32_t width) {
    KernelFn k = pick(kind, strategy, width);
    if (!k) return 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, (int)width, 0) != hipSuccess) return 0;
    return n;
}

}  // namespace rs

// ---------------------------------------------------------------- region validation

namespace rs {

// Checks borrowed device regions before any pipeline kernel reads through them:
// CSR offsets non-decreasing and within the element array, or start+length regions
// in order, disjoint and within the array.  Records the first bad parent.
__global__ void validate_regions(const uint32_t *offs, const uint32_t *lens, uint32_t P, uint32_t n,
                                 uint32_t *bad) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    bool ok;
    if (!lens) {
        ok = offs[i] <= offs[i + 1] && offs[i + 1] <= n;
    } else {
        const unsigned long long end = (unsigned long long)offs[i] + lens[i];
        ok = end <= n && (i + 1 == P || end <= offs[i + 1]);
    }
    if (!ok) atomicMin(bad, i);
}

int validate_device_regions(const uint32_t *offs, const uint32_t *lens, uint32_t P, uint32_t n, void *stream) {
    uint32_t *bad = nullptr;
    hipError_t e = hipMalloc(&bad, 4);
    if (e != hipSuccess) return -(int)e;
    uint32_t h = 0xFFFFFFFFu;
    e = hipMemcpyAsync(bad, &h, 4, hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(validate_regions, dim3((P + 255) / 256), dim3(256), 0, (hipStream_t)stream, offs, lens, P,
                           n, bad);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(bad);
    if (e != hipSuccess) return -(int)e;
    return h == 0xFFFFFFFFu ? 0 : (int)(h + 1u);
}

}  // namespace rs
