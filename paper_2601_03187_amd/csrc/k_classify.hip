// Search stage of the two-stage classification (Sec. 5.1.1), one packet per lane:
//   1. probe the predicted tuples: truncate SIP/DIP to the tuple's prefix lengths,
//      hash, walk the open-addressing slots to the bucket, and compare the bucket's
//      rules one by one in (priority, id) order -- the first match is the bucket's best;
//   2. certify: if a rule matched, probe the tuples of its conflict mask (the only
//      tuples that can hold a better matching rule); if nothing matched, probe every
//      remaining tuple (the paper's post-verification search, Sec. 5.1.1); in both
//      cases a tuple whose best (lowest) key cannot beat the current answer is skipped.
// Before any slot walk, a bit of the bucket filter rules out a tuple that has no bucket
// for the header's masked addresses. The filter is blocked by prefix group (the tuples
// sharing their longer field's length): one 8-byte block answers every tuple of its
// group, so certification loads one block per group it needs -- all of them at once,
// eight independent loads at a time -- and then each lane walks slots only for its own
// tuples whose bit is set. Random loads are what the search pays for (each one costs
// an L2 request whatever its width), so the scan also reads only the first half of each
// record and the second half only when a rule matches.
// Candidates come packed in the output word from the MLP (one byte per candidate, 16
// bits above 256 tuples). Tuple spaces of more than 32 tuples use the same steps over
// multiword tuple masks (8 words up to 256 tuples, 16 up to 512), with conflict masks in
// a side array.
#include <type_traits>

#include "tang_internal.hpp"

namespace tang {
namespace {

constexpr uint32_t kNoTuple = 0xFFFFFFFFu;

struct Best {
    uint32_t prio, id, cmask, tuple, pos;   // pos: record index (for wide conflict masks)
};

__device__ __forceinline__ bool kless(uint32_t p1, uint32_t i1, uint32_t p2, uint32_t i2) {
    return p1 < p2 || (p1 == p2 && i1 < i2);
}

// Whole 16-byte loads. Copying the structs field by field lets the compiler split them
// into narrow loads sunk into the branches that use each field: more load instructions
// per wave and dependent round trips between them. An empty asm that takes all four
// words keeps each 16-byte load whole and in place.
__device__ __forceinline__ uint4 load16(const void* p) {
    uint4 a = *reinterpret_cast<const uint4*>(p);
    asm volatile("" : "+v"(a.x), "+v"(a.y), "+v"(a.z), "+v"(a.w));
    return a;
}
__device__ __forceinline__ Slot load_slot(const Slot* p) {
    const uint4 a = load16(p);
    return Slot{a.x, a.y, a.z, a.w};
}
__device__ __forceinline__ uint2 load8(const uint2* p) {
    uint2 a = *p;
    asm volatile("" : "+v"(a.x), "+v"(a.y));
    return a;
}

// Compares one list of records in (priority, id) order: the first match is its best;
// the scan stops there or at the first record that cannot beat the current answer.
// The hot half (ports, priority, protocol/lengths) decides; the cold half (prefixes,
// id, conflict mask) is read for a priority tie, a rule held by a coarser tuple, and
// the match.
template <bool STATS>
__device__ __forceinline__ void scan_list(uint32_t t, uint32_t off, uint32_t len, uint32_t sip,
                                          uint32_t dip, uint32_t sp, uint32_t dp, uint32_t proto,
                                          const Rec* __restrict__ recs, Best& b, uint32_t& n_recs) {
    for (uint32_t k = 0; k < len; ++k) {
        const uint4* p = reinterpret_cast<const uint4*>(recs + off + k);
        const uint4 h = load16(p);  // sp, dp, prio, meta
        if (STATS) ++n_recs;
        if (h.z > b.prio) break;
        const bool ok = ((uint32_t)(sp >= (h.x & 0xFFFFu)) & (uint32_t)(sp <= (h.x >> 16)) &
                         (uint32_t)(dp >= (h.y & 0xFFFFu)) & (uint32_t)(dp <= (h.y >> 16)) &
                         ((uint32_t)(meta_exact(h.w) == 0) | (uint32_t)(proto == meta_proto(h.w)))) != 0u;
        if (!ok && h.z < b.prio) continue;
        const uint4 c = load16(p + 1);  // sip, dip, id, cmask
        if (h.z == b.prio && !(c.z < b.id)) break;
        if (!ok) continue;
        if (meta_check(h.w)) {
            const uint32_t sm = pmask(meta_sl(h.w)), dm = pmask(meta_dl(h.w));
            if (((sip ^ c.x) & sm) | ((dip ^ c.y) & dm)) continue;
        }
        b = Best{h.z, c.z, c.w, t, off + k};
        break;
    }
}

// Walks the open-addressing slots from hash h to key (tk, k0, k1); returns the slot, or
// an empty one. The table is kept at most a third full, so an empty slot ends every
// walk; the step bound only guards against a corrupted table.
template <bool STATS>
__device__ __forceinline__ Slot find_slot(uint64_t h64, uint32_t tk, uint32_t k0, uint32_t k1,
                                          uint32_t slot_mask, const Slot* __restrict__ slots,
                                          uint32_t& n_slots) {
    uint32_t h = slot_of(h64) & slot_mask;
    for (uint32_t step = 0; step <= slot_mask; ++step) {
        const Slot s = load_slot(slots + h);
        if (STATS) ++n_slots;
        if (s.tl == kEmptyTL || (s.ms == k0 && s.md == k1 && (s.tl >> kTlShift) == tk)) return s;
        h = (h + 1) & slot_mask;
    }
    return Slot{0, 0, kEmptyTL, 0};
}

// Searches tuple t for this header: the slot walk to the bucket, then the bucket's list,
// or for a split bucket the sub-lists the header selects.
template <bool STATS>
__device__ __forceinline__ void search_tuple(uint32_t t, const TupleDev* s_t, uint32_t sip,
                                             uint32_t dip, uint32_t sp, uint32_t dp, uint32_t proto,
                                             uint32_t slot_mask, const Slot* __restrict__ slots,
                                             const Rec* __restrict__ recs, Best& b,
                                             uint32_t& n_probe, uint32_t& n_slots, uint32_t& n_recs) {
    if (STATS) ++n_probe;
    const uint32_t ms = sip & s_t[t].smask, md = dip & s_t[t].dmask;
    const Slot s = find_slot<STATS>(key_hash(t, ms, md), t, ms, md, slot_mask, slots, n_slots);
    if (s.tl == kEmptyTL) return;
    if (!(s.off & kSplit)) {
        scan_list<STATS>(t, s.off, s.tl & kMaxBucketLen, sip, dip, sp, dp, proto, recs, b, n_recs);
        return;
    }
    // a split bucket: only the four sub-lists this header's DP, SP and protocol select
    const uint32_t bi = s.off & ~kSplit;
    const uint32_t keys[4][2] = {{kSubDp, dp}, {kSubSp, sp}, {kSubProto, proto}, {kSubRest, 0u}};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t tk = t | (keys[q][0] << kKindShift);
        const Slot u = find_slot<STATS>(key_hash(tk, bi, keys[q][1]), tk, bi, keys[q][1], slot_mask,
                                        slots, n_slots);
        if (u.tl != kEmptyTL)
            scan_list<STATS>(t, u.off, u.tl & kMaxBucketLen, sip, dip, sp, dp, proto, recs, b, n_recs);
    }
}

// The filter block of group key gk for this header.
__device__ __forceinline__ const uint2* block_of(const uint2* __restrict__ filter, uint32_t gk,
                                                 uint32_t sip, uint32_t dip, uint32_t filter_mask) {
    const uint32_t len = gk & 63u;
    const uint32_t v = (gk & 64u ? dip : sip) & pmask(len);
    return filter + (filter_block(gk, v) & filter_mask);
}

// Whether tuple t of group key gk may hold a bucket for this header, given its block.
__device__ __forceinline__ bool block_has(uint2 blk, uint32_t t, uint32_t gk, const TupleDev* s_t,
                                          uint32_t sip, uint32_t dip) {
    const uint32_t o = gk & 64u ? (sip & s_t[t].smask) : (dip & s_t[t].dmask);
    const uint32_t bits = filter_bits(t, o), b1 = bits & 63u, b2 = bits >> 8;
    return ((b1 & 32u ? blk.y : blk.x) >> (b1 & 31u)) & ((b2 & 32u ? blk.y : blk.x) >> (b2 & 31u)) & 1u;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor(v, o, 64));
    return v;
}

// OR of a 32-bit mask over the wave, as a wave-uniform value.
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// NW: conflict-mask words (1 for at most 32 tuples, kMaskWords for up to 256, kMaxWords
// above). Tuple sets are NW-word bit masks (word t / 32, bit t % 32); group sets one
// word (at most 32 groups) or two (64). The best-key prefixes stay in LDS up to 256
// tuples; above, the one row a lane needs is read from the tuple table.
template <bool STATS, int NW>
__global__ __launch_bounds__(256) void k_classify(const uint4* __restrict__ hdr,
                                                  uint32_t* __restrict__ out, uint32_t n,
                                                  const Slot* __restrict__ slots,
                                                  const Rec* __restrict__ recs,
                                                  const uint32_t* __restrict__ cmask_rows,
                                                  const uint2* __restrict__ filter,
                                                  const TupleTable* __restrict__ ttg, int kcand,
                                                  StatsDev* __restrict__ st,
                                                  const uint32_t* __restrict__ live) {
    constexpr uint32_t NT = 32u * NW;
    constexpr int NG = NW == 1 ? 32 : kMaxGroups;   // groups: at most one per tuple
    constexpr bool PREFIX_LDS = NW <= kMaskWords;
    constexpr uint32_t CB = NW > kMaskWords ? 16u : 8u;   // bits per packed candidate
    using GMask = typename std::conditional<NW == 1, uint32_t, unsigned long long>::type;
    __shared__ TupleDev s_t[NT];
    __shared__ uint2 s_rank[NT];  // best keys in ascending order
    __shared__ uint32_t s_prefix[PREFIX_LDS ? NT + 1 : 1][NW];
    __shared__ uint32_t s_all[NW], s_nog[NW];
    __shared__ uint32_t s_gid[NT];
    __shared__ uint32_t s_gkey[NG];
    __shared__ uint32_t s_gmask[NG][NW];
    __shared__ uint32_t s_misc[4];
    const int tid = threadIdx.x;
    if (live) n = min(n, *live);
    if (blockIdx.x * 256u >= n) return;   // uniform over the block (a live count below the grid)
    for (uint32_t k = tid; k < NT; k += 256u) {
        s_t[k] = ttg->t[k];
        s_rank[k] = make_uint2(ttg->rank_prio[k], ttg->rank_id[k]);
        s_gid[k] = ttg->gid[k];
    }
    if constexpr (PREFIX_LDS)
        for (uint32_t k = tid; k < (NT + 1) * NW; k += 256u) s_prefix[k / NW][k % NW] = ttg->prefix[k / NW][k % NW];
    for (uint32_t k = tid; k < (uint32_t)NG * NW; k += 256u) s_gmask[k / NW][k % NW] = ttg->gmask[k / NW][k % NW];
    if (tid < NG) s_gkey[tid] = ttg->gkey[tid];
    if (tid < NW) {
        s_all[tid] = ttg->all_mask[tid];
        s_nog[tid] = ttg->nogroup[tid];
    }
    if (tid == 0) {
        s_misc[0] = ttg->n;
        s_misc[1] = ttg->ngroups;
        s_misc[2] = ttg->slot_mask;
        s_misc[3] = ttg->filter_mask;
    }
    __syncthreads();
    const uint32_t ntup = s_misc[0], ngroups = s_misc[1], slot_mask = s_misc[2], filter_mask = s_misc[3];
    const uint32_t i = blockIdx.x * 256u + tid;
    uint32_t n_probe = 0, n_slots = 0, n_recs = 0, top1 = 0, fb = 0, nm = 0, active = 0;
    uint32_t n_filter = 0, n_steps = 0, n_rounds = 0;
    uint32_t sip = 0, dip = 0, sp = 0, dp = 0, proto = 0, c0 = kNoTuple;
    uint32_t todo[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) todo[w] = 0;
    Best b{kDead, kDead, 0u, 0u, 0u};
    // the first candidate's group block, kept for the other tuples of its group
    uint32_t g0 = kNoGroup;
    uint2 blk0 = make_uint2(0u, 0u);
    if (i < n) {
        active = 1;
        const uint4 h = hdr[i];
        sip = h.x;
        dip = h.y;
        sp = h.z & 0xFFFFu;
        dp = h.z >> 16;
        proto = h.w & 0xFFu;
        bool found = false;
        uint32_t probed[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) probed[w] = 0;
        if (kcand > 0) {
            const uint32_t cp = out[i];
            for (int c = 0; c < kcand; ++c) {
                const uint32_t t = (cp >> (CB * c)) & ((1u << CB) - 1u);
                if (c == 0) c0 = t;
                if (t >= ntup) continue;
                uint32_t& pw = probed[NW == 1 ? 0 : t >> 5];
                if ((pw >> (t & 31u)) & 1u) continue;
                pw |= 1u << (t & 31u);
                if (!kless(s_t[t].best_prio, s_t[t].best_id, b.prio, b.id)) continue;
                const uint32_t g = s_gid[t];
                bool pass = true;
                if (g != kNoGroup) {
                    const uint32_t gk = s_gkey[g];
                    uint2 blk;
                    if (g == g0) {
                        blk = blk0;
                    } else {
                        blk = load8(block_of(filter, gk, sip, dip, filter_mask));
                        if (STATS) ++n_filter;
                    }
                    if (g0 == kNoGroup) {
                        g0 = g;
                        blk0 = blk;
                    }
                    pass = block_has(blk, t, gk, s_t, sip, dip);
                }
                if (pass)
                    search_tuple<STATS>(t, s_t, sip, dip, sp, dp, proto, slot_mask, slots, recs, b,
                                        n_probe, n_slots, n_recs);
            }
            found = b.id != kDead;
        }
        if (NW == 1 || !found) {
#pragma unroll
            for (int w = 0; w < NW; ++w)
                todo[w] = (found ? b.cmask : s_all[w]) & ~probed[w] & s_all[w];
        } else {
            const uint4* row = reinterpret_cast<const uint4*>(cmask_rows + (size_t)b.pos * NW);
#pragma unroll
            for (int q = 0; q < NW / 4; ++q) {
                const uint4 m = row[q];
                todo[4 * q] = m.x & ~probed[4 * q];
                todo[4 * q + 1] = m.y & ~probed[4 * q + 1];
                todo[4 * q + 2] = m.z & ~probed[4 * q + 2];
                todo[4 * q + 3] = m.w & ~probed[4 * q + 3];
            }
        }
        if (STATS) fb = found ? 0u : 1u;
    }
    // Certification. First drop the tuples whose best key cannot beat the answer: the
    // tuples in ascending best-key order form a prefix, found by a binary search.
    {
        uint32_t any = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) any |= todo[w];
        if (any) {
            uint32_t k = 0;
#pragma unroll
            for (uint32_t step = NT; step > 0; step >>= 1)
                if (k + step <= ntup && kless(s_rank[k + step - 1].x, s_rank[k + step - 1].y, b.prio, b.id))
                    k += step;
            if constexpr (PREFIX_LDS) {
#pragma unroll
                for (int w = 0; w < NW; ++w) todo[w] &= s_prefix[k][w];
            } else {
                const uint4* row = reinterpret_cast<const uint4*>(ttg->prefix[k]);
#pragma unroll
                for (int q = 0; q < NW / 4; ++q) {
                    const uint4 m = row[q];
                    todo[4 * q] &= m.x;
                    todo[4 * q + 1] &= m.y;
                    todo[4 * q + 2] &= m.z;
                    todo[4 * q + 3] &= m.w;
                }
            }
        }
    }
    // Phase 1: the groups the remaining tuples need (the first candidate's block is
    // already here), their blocks eight at a time per lane, then each needed tuple's bit.
    uint32_t hits[NW];
    GMask gneed = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) hits[w] = todo[w] & s_nog[w];
    if (g0 != kNoGroup) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            for (uint32_t m = todo[w] & s_gmask[g0][w]; m; m &= m - 1u) {
                const uint32_t t = 32u * w + (uint32_t)__builtin_ctz(m);
                if (block_has(blk0, t, s_gkey[g0], s_t, sip, dip)) hits[w] |= 1u << (t & 31u);
            }
        }
    }
    {
        uint32_t any = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) any |= todo[w];
        if (wave_or(any)) {
            for (uint32_t g = 0; g < ngroups; ++g) {
                uint32_t m = 0;
#pragma unroll
                for (int w = 0; w < NW; ++w) m |= todo[w] & s_gmask[g][w];
                if (m && g != g0) gneed |= (GMask)1 << g;
            }
        }
    }
    for (;;) {
        if (!wave_or(gneed != 0 ? 1u : 0u)) break;
        if (STATS) ++n_rounds;
        uint32_t gq[8];
        uint2 blk[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            gq[q] = kNoGroup;
            blk[q] = make_uint2(0u, 0u);
            if (gneed) {
                const uint32_t g = NW == 1 ? (uint32_t)__builtin_ctz((uint32_t)gneed)
                                           : (uint32_t)__builtin_ctzll((unsigned long long)gneed);
                gneed &= gneed - 1;
                gq[q] = g;
                blk[q] = load8(block_of(filter, s_gkey[g], sip, dip, filter_mask));
                if (STATS) ++n_filter;
            }
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (gq[q] == kNoGroup) continue;
            const uint32_t gk = s_gkey[gq[q]];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                for (uint32_t m = todo[w] & s_gmask[gq[q]][w]; m; m &= m - 1u) {
                    const uint32_t t = 32u * w + (uint32_t)__builtin_ctz(m);
                    if (block_has(blk[q], t, gk, s_t, sip, dip)) hits[w] |= 1u << (t & 31u);
                }
            }
        }
    }
    // Phase 2: each lane searches its own passing tuples in tuple order -- tuples are
    // numbered by first appearance in priority order, so good answers come early --
    // skipping any whose best key can no longer beat the answer. The probes run as one
    // flat loop of loads per lane (slot, record first half, record second half; a lane
    // between probes takes its next tuple at the top of the loop), so a wave takes as
    // many iterations as its busiest lane issues loads in total. Probe by probe in
    // lockstep, a wave would wait at every probe for its lane with the longest walk or
    // bucket scan, and lanes with long scans rarely coincide.
    uint32_t steps = 0;
    {
        enum : uint32_t { P_NEXT = 0, P_SLOT, P_HOT, P_COLD, P_DONE };
        constexpr uint32_t kMain = 8;   // `sub` while walking to a tuple's main bucket
        uint32_t ps = active ? P_NEXT : P_DONE;
        uint32_t ct = 0, tk = 0, k0 = 0, k1 = 0, walk = 0, sub = kMain, bi = 0, left = 0;
        uint32_t hp = 0, hm = 0, hok = 0;
        const uint4* ld = reinterpret_cast<const uint4*>(slots);
        for (;;) {
            if (ps == P_NEXT) {
                ps = P_DONE;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    while (hits[w]) {
                        const uint32_t t = 32u * w + (uint32_t)__builtin_ctz(hits[w]);
                        hits[w] &= hits[w] - 1u;
                        if (kless(s_t[t].best_prio, s_t[t].best_id, b.prio, b.id)) {
                            ct = t;
                            ps = P_SLOT;
                            break;
                        }
                    }
                    if (ps == P_SLOT) break;
                }
                if (ps == P_SLOT) {
                    if (STATS) ++n_probe;
                    tk = ct;
                    k0 = sip & s_t[ct].smask;
                    k1 = dip & s_t[ct].dmask;
                    sub = kMain;
                    walk = 0;
                    ld = reinterpret_cast<const uint4*>(slots + (slot_of(key_hash(tk, k0, k1)) & slot_mask));
                }
            }
            if (!__ballot(ps != P_DONE)) break;
            if (STATS && ps != P_DONE) ++steps;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (ps != P_DONE) v = load16(ld);
            bool list_done = false;
            if (ps == P_SLOT) {
                if (STATS) ++n_slots;
                if (v.z == kEmptyTL) {
                    list_done = true;
                } else if (v.x == k0 && v.y == k1 && (v.z >> kTlShift) == tk) {
                    if (sub == kMain && (v.w & kSplit)) {
                        bi = v.w & ~kSplit;   // a split bucket: the sub-lists the header selects
                        sub = 0;
                        list_done = true;
                    } else if ((v.z & kMaxBucketLen) == 0) {
                        list_done = true;
                    } else {
                        left = (v.z & kMaxBucketLen) - 1u;
                        ps = P_HOT;
                        ld = reinterpret_cast<const uint4*>(recs + v.w);
                    }
                } else if (++walk > slot_mask) {
                    list_done = true;   // only a corrupted table has no empty slot
                } else {
                    const uint32_t h = (uint32_t)(reinterpret_cast<const Slot*>(ld) - slots);
                    ld = reinterpret_cast<const uint4*>(slots + ((h + 1u) & slot_mask));
                }
            } else if (ps == P_HOT) {
                if (STATS) ++n_recs;
                if (v.z > b.prio) {
                    list_done = true;   // this and every later record cannot beat the answer
                } else {
                    const bool ok = ((uint32_t)(sp >= (v.x & 0xFFFFu)) & (uint32_t)(sp <= (v.x >> 16)) &
                                     (uint32_t)(dp >= (v.y & 0xFFFFu)) & (uint32_t)(dp <= (v.y >> 16)) &
                                     ((uint32_t)(meta_exact(v.w) == 0) |
                                      (uint32_t)(proto == meta_proto(v.w)))) != 0u;
                    if (!ok && v.z < b.prio) {
                        if (left) {
                            --left;
                            ld += 2;
                        } else {
                            list_done = true;
                        }
                    } else {
                        hp = v.z;
                        hm = v.w;
                        hok = ok ? 1u : 0u;
                        ps = P_COLD;
                        ld += 1;
                    }
                }
            } else if (ps == P_COLD) {
                bool next = false;
                if (hp == b.prio && !(v.z < b.id)) {
                    list_done = true;
                } else if (!hok) {
                    next = true;
                } else if (meta_check(hm) && ((((sip ^ v.x) & pmask(meta_sl(hm))) |
                                               ((dip ^ v.y) & pmask(meta_dl(hm)))) != 0u)) {
                    next = true;
                } else {
                    b = Best{hp, v.z, v.w, ct, (uint32_t)(reinterpret_cast<const Rec*>(ld - 1) - recs)};
                    list_done = true;
                }
                if (next) {
                    if (left) {
                        --left;
                        ps = P_HOT;
                        ld += 1;
                    } else {
                        list_done = true;
                    }
                }
            }
            if (list_done) {
                if (sub < 4u) {
                    // the next sub-list of a split bucket
                    const uint32_t kind = sub == 0 ? kSubDp : sub == 1 ? kSubSp : sub == 2 ? kSubProto : kSubRest;
                    const uint32_t val = sub == 0 ? dp : sub == 1 ? sp : sub == 2 ? proto : 0u;
                    ++sub;
                    tk = ct | (kind << kKindShift);
                    k0 = bi;
                    k1 = val;
                    walk = 0;
                    ps = P_SLOT;
                    ld = reinterpret_cast<const uint4*>(slots + (slot_of(key_hash(tk, k0, k1)) & slot_mask));
                } else {
                    ps = P_NEXT;
                }
            }
        }
    }
    if (STATS) n_steps = wave_max(steps);
    if (active) {
        const bool found = b.id != kDead;
        out[i] = found ? b.id : TANG_NO_MATCH;
        if (STATS) {
            top1 = (found && b.tuple == c0) ? 1u : 0u;
            nm = found ? 0u : 1u;
        }
    }
    if (STATS) {
        // wave sums -> block sums in LDS -> one set of atomics per block, spread over
        // kStatCopies counter copies (summed on the host) to avoid one hot address
        constexpr int NS = 10;
        __shared__ unsigned long long s_red[4][NS];
        unsigned long long v[NS] = {active, n_probe, n_slots, n_recs, top1, fb, nm, n_filter,
                                    active ? n_steps : 0u, active ? n_rounds : 0u};
#pragma unroll
        for (int q = 0; q < NS; ++q) v[q] = wave_sum(v[q]);
        if ((tid & 63) == 0)
#pragma unroll
            for (int q = 0; q < NS; ++q) s_red[tid >> 6][q] = v[q];
        __syncthreads();
        if (tid < NS) {
            const unsigned long long sum = s_red[0][tid] + s_red[1][tid] + s_red[2][tid] + s_red[3][tid];
            unsigned long long* dst = reinterpret_cast<unsigned long long*>(st + (blockIdx.x % kStatCopies));
            atomicAdd(dst + tid, sum);
        }
    }
}

}  // namespace

hipError_t launch_classify(const tang_ruleset_t* rs, const tang_header_t* d_hdr, uint32_t* d_out,
                           size_t n, int kcand, hipStream_t s, bool stats, const uint32_t* d_live) {
    const size_t chunk = (size_t)1 << 30;
    if (d_live && n > chunk) return hipErrorInvalidValue;
    for (size_t base = 0; base < n; base += chunk) {
        const uint32_t m = (uint32_t)std::min(chunk, n - base);
        const dim3 grid((m + 255) / 256), block(256);
        const uint4* h = reinterpret_cast<const uint4*>(d_hdr) + base;
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, block, 0, s, h, d_out + base, m, rs->d_slots, rs->d_recs,
                               rs->d_cmask, reinterpret_cast<const uint2*>(rs->d_filter), rs->d_tt,
                               kcand, rs->d_stats, d_live);
        };
        if (rs->nw == 1) {
            if (stats) go(k_classify<true, 1>);
            else go(k_classify<false, 1>);
        } else if (rs->nw == kMaskWords) {
            if (stats) go(k_classify<true, kMaskWords>);
            else go(k_classify<false, kMaskWords>);
        } else {
            if (stats) go(k_classify<true, kMaxWords>);
            else go(k_classify<false, kMaxWords>);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tang
