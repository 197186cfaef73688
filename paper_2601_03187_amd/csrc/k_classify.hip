// Search stage of the two-stage classification (Sec. 5.1.1), one packet per lane:
//   1. probe the predicted tuples: truncate SIP/DIP to the tuple's prefix lengths,
//      hash, walk the open-addressing slots to the bucket, and compare the bucket's
//      rules one by one in (priority, id) order -- the first match is the bucket's best;
//   2. certify: if a rule matched, probe the tuples of its conflict mask (the only
//      tuples that can hold a better matching rule); if nothing matched, probe every
//      remaining tuple (the paper's post-verification search, Sec. 5.1.1); in both
//      cases a tuple whose best (lowest) key cannot beat the current answer is skipped.
// Before any slot walk, a bit of the bucket filter rules out a tuple that has no bucket
// for the header's masked addresses. Certification first sweeps the filter for all of a
// packet's remaining tuples, eight independent loads at a time, and then each lane walks
// slots only for its own tuples whose bit is set. Both halves matter on a 64-lane wave:
// one dependent L2 round trip per tuple would cost two dozen round trips back to back,
// and a wave-uniform loop over tuples would pay for the union of all lanes' tuples.
// Candidates come packed in the output word (one byte per candidate) from the MLP.
// Tuple spaces of more than 32 tuples (up to 256) use the same steps over eight-word
// tuple masks, with conflict masks in a side array, a pre-check of the header's field
// keys before the filter sweep, and per-lane filter batches.
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

__device__ __forceinline__ bool rec_match(const Rec& r, uint32_t sip, uint32_t dip, uint32_t sp,
                                          uint32_t dp, uint32_t proto) {
    const uint32_t m = r.meta;
    const uint32_t sm = pmask(meta_sl(m)), dm = pmask(meta_dl(m));
    bool ok = (((sip ^ r.sip) & sm) == 0) & (((dip ^ r.dip) & dm) == 0);
    ok &= (sp >= (r.sp & 0xFFFFu)) & (sp <= (r.sp >> 16));
    ok &= (dp >= (r.dp & 0xFFFFu)) & (dp <= (r.dp >> 16));
    ok &= (meta_exact(m) == 0) | (proto == meta_proto(m));
    return ok;
}

// Whole-record and whole-slot loads (two and one 16-byte loads). Copying the structs
// field by field lets the compiler split them into narrow loads sunk into the branches
// that use each field: more load instructions per wave and dependent round trips
// between them (priority and id first, the rest after the comparison).
// An empty asm that takes all four words keeps each 16-byte load whole and in place.
__device__ __forceinline__ uint4 load16(const void* p) {
    uint4 a = *reinterpret_cast<const uint4*>(p);
    asm volatile("" : "+v"(a.x), "+v"(a.y), "+v"(a.z), "+v"(a.w));
    return a;
}
__device__ __forceinline__ Rec load_rec(const Rec* p) {
    const uint4 a = load16(p), c = load16(reinterpret_cast<const uint4*>(p) + 1);
    return Rec{a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w};
}
__device__ __forceinline__ Slot load_slot(const Slot* p) {
    const uint4 a = load16(p);
    return Slot{a.x, a.y, a.z, a.w};
}

// Compares one list of records in (priority, id) order: the first match is its best;
// the scan stops there or at the first record that cannot beat the current answer.
template <bool STATS>
__device__ __forceinline__ void scan_list(uint32_t off, uint32_t len, uint32_t sip, uint32_t dip,
                                          uint32_t sp, uint32_t dp, uint32_t proto,
                                          const Rec* __restrict__ recs, Best& b, uint32_t& n_recs) {
    for (uint32_t k = 0; k < len; ++k) {
        const Rec r = load_rec(recs + off + k);
        if (STATS) ++n_recs;
        if (!kless(r.prio, r.id, b.prio, b.id)) break;
        if (rec_match(r, sip, dip, sp, dp, proto)) {
            b = Best{r.prio, r.id, r.cmask, meta_tuple(r.meta), off + k};
            break;
        }
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

// Searches tuple t for this header (its masked key and hash given): the slot walk to the
// bucket, then the bucket's list, or for a split bucket the sub-lists the header selects.
template <bool STATS>
__device__ __forceinline__ void search_tuple(uint32_t t, uint64_t h, uint32_t ms, uint32_t md,
                                             uint32_t sip, uint32_t dip, uint32_t sp, uint32_t dp,
                                             uint32_t proto, uint32_t slot_mask,
                                             const Slot* __restrict__ slots,
                                             const Rec* __restrict__ recs, Best& b,
                                             uint32_t& n_probe, uint32_t& n_slots, uint32_t& n_recs) {
    if (STATS) ++n_probe;
    const Slot s = find_slot<STATS>(h, t, ms, md, slot_mask, slots, n_slots);
    if (s.tl == kEmptyTL) return;
    if (!(s.off & kSplit)) {
        scan_list<STATS>(s.off, s.tl & kMaxBucketLen, sip, dip, sp, dp, proto, recs, b, n_recs);
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
            scan_list<STATS>(u.off, u.tl & kMaxBucketLen, sip, dip, sp, dp, proto, recs, b, n_recs);
    }
}

// Searches tuple t for this header after checking its filter bit.
template <bool STATS>
__device__ __forceinline__ void probe(uint32_t t, uint32_t sip, uint32_t dip, uint32_t sp,
                                      uint32_t dp, uint32_t proto, const TupleDev* s_t,
                                      uint32_t slot_mask, uint32_t filter_mask,
                                      const uint32_t* __restrict__ filter,
                                      const Slot* __restrict__ slots, const Rec* __restrict__ recs,
                                      Best& b, uint32_t& n_probe, uint32_t& n_slots,
                                      uint32_t& n_recs, uint32_t& n_filter) {
    const uint32_t ms = sip & s_t[t].smask, md = dip & s_t[t].dmask;
    const uint32_t bit = filter_hash(t, ms, md) & filter_mask;
    if (STATS) ++n_filter;
    if (!((filter[bit >> 5] >> (bit & 31u)) & 1u)) return;
    search_tuple<STATS>(t, key_hash(t, ms, md), ms, md, sip, dip, sp, dp, proto, slot_mask, slots,
                        recs, b, n_probe, n_slots, n_recs);
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

// NW: conflict-mask words (1 for at most 32 tuples, kMaskWords for up to 256). Tuple
// sets are NW-word bit masks (word t / 32, bit t % 32); everything else is as for one word.
template <bool STATS, int NW, bool RANKED>
__global__ __launch_bounds__(256) void k_classify(const uint4* __restrict__ hdr,
                                                  uint32_t* __restrict__ out, uint32_t n,
                                                  const Slot* __restrict__ slots,
                                                  const Rec* __restrict__ recs,
                                                  const uint32_t* __restrict__ cmask_rows,
                                                  const uint32_t* __restrict__ filter,
                                                  const TupleTable* __restrict__ ttg, int kcand,
                                                  StatsDev* __restrict__ st) {
    constexpr uint32_t NT = 32u * NW;
    __shared__ TupleDev s_t[NT];
    __shared__ uint2 s_rank[NT];  // best keys in ascending order
    __shared__ uint32_t s_order[NT];  // tuple indices in that order
    __shared__ uint32_t s_prefix[NT + 1][NW];
    __shared__ uint32_t s_all[NW];
    __shared__ uint32_t s_misc[4];
    // field pre-check (wide tuple spaces only): distinct lengths and their tuple masks
    constexpr int NF = NW > 1 ? 33 : 1;
    __shared__ uint32_t s_flen[2][NF];
    __shared__ uint32_t s_fmask[2][NF][NW];
    __shared__ uint32_t s_nflen[2];
    const int tid = threadIdx.x;
    for (uint32_t k = tid; k < NT; k += 256u) {
        s_t[k] = ttg->t[k];
        s_rank[k] = make_uint2(ttg->rank_prio[k], ttg->rank_id[k]);
        s_order[k] = ttg->order[k];
    }
    for (uint32_t k = tid; k < (NT + 1) * NW; k += 256u) s_prefix[k / NW][k % NW] = ttg->prefix[k / NW][k % NW];
    if (tid < NW) s_all[tid] = ttg->all_mask[tid];
    if constexpr (NW > 1) {
        for (uint32_t k = tid; k < 2u * NF * NW; k += 256u)
            s_fmask[k / (NF * NW)][(k / NW) % NF][k % NW] = ttg->fmask[k / (NF * NW)][(k / NW) % NF][k % NW];
        if (tid < 2 * NF) s_flen[tid / NF][tid % NF] = ttg->flen[tid / NF][tid % NF];
        if (tid < 2) s_nflen[tid] = ttg->nflen[tid];
    }
    if (tid == 0) {
        s_misc[0] = ttg->n;
        s_misc[2] = ttg->slot_mask;
        s_misc[3] = ttg->filter_mask;
    }
    __syncthreads();
    const uint32_t ntup = s_misc[0], slot_mask = s_misc[2], filter_mask = s_misc[3];
    const uint32_t i = blockIdx.x * 256u + tid;
    uint32_t n_probe = 0, n_slots = 0, n_recs = 0, top1 = 0, fb = 0, nm = 0, active = 0;
    uint32_t n_filter = 0, n_steps = 0, n_rounds = 0;
    uint32_t sip = 0, dip = 0, sp = 0, dp = 0, proto = 0, c0 = kNoTuple;
    uint32_t todo[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) todo[w] = 0;
    Best b{kDead, kDead, 0u, 0u, 0u};
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
                const uint32_t t = (cp >> (8 * c)) & 0xFFu;
                if (c == 0) c0 = t;
                if (t >= ntup) continue;
                uint32_t& pw = probed[NW == 1 ? 0 : t >> 5];
                if ((pw >> (t & 31u)) & 1u) continue;
                pw |= 1u << (t & 31u);
                if (!kless(s_t[t].best_prio, s_t[t].best_id, b.prio, b.id)) continue;
                probe<STATS>(t, sip, dip, sp, dp, proto, s_t, slot_mask, filter_mask, filter, slots,
                             recs, b, n_probe, n_slots, n_recs, n_filter);
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
#pragma unroll
            for (int w = 0; w < NW; ++w) todo[w] &= s_prefix[k][w];
        }
    }
    // Wide tuple spaces, headers with many tuples left (all that matched nothing yet, and
    // those with a wide conflict mask): check the field keys of the distinct lengths of
    // each field (eight loads at a time) and keep only the tuples whose SIP and DIP
    // lengths both passed. Below 25 tuples three more batches would not pay.
    if constexpr (NW > 1) {
        uint32_t left = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) left += __builtin_popcount(todo[w]);
        const bool many = left > 24u;
        if (wave_or(many ? 1u : 0u)) {
            unsigned long long pass[2] = {0ull, 0ull};
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const uint32_t nl = s_nflen[side], v = side == 0 ? sip : dip;
                for (uint32_t i0 = 0; i0 < nl; i0 += 8) {
                    if (STATS) ++n_rounds;
                    uint32_t wd[8], pos[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        wd[q] = 0;
                        pos[q] = 0;
                        if (many && i0 + q < nl) {
                            const uint32_t len = s_flen[side][i0 + q];
                            const uint32_t bit = field_filter_hash(side, len, v & pmask(len)) & filter_mask;
                            wd[q] = filter[bit >> 5];
                            pos[q] = bit & 31u;
                            if (STATS) ++n_filter;
                        }
                    }
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        pass[side] |= (unsigned long long)((wd[q] >> pos[q]) & 1u) << (i0 + q);
                }
            }
            if (many) {
                uint32_t keep[2][NW];
#pragma unroll
                for (int side = 0; side < 2; ++side) {
#pragma unroll
                    for (int w = 0; w < NW; ++w) keep[side][w] = 0;
                    for (unsigned long long m = pass[side]; m; m &= m - 1ull) {
                        const uint32_t j = (uint32_t)__builtin_ctzll(m);
#pragma unroll
                        for (int w = 0; w < NW; ++w) keep[side][w] |= s_fmask[side][j][w];
                    }
                }
#pragma unroll
                for (int w = 0; w < NW; ++w) todo[w] &= keep[0][w] & keep[1][w];
            }
        }
    }
    uint32_t steps = 0;
    if constexpr (RANKED) {
        // Without candidates (no model), one mask word: the tuples go in rank order
        // (ascending best key), eight ranks per batch -- the filter bits of the batch's
        // tuples this lane still needs, eight loads issued back to back, then this lane's
        // probes of the passing ones. A tuple is needed while its best key beats the
        // answer, so an answer found in an early batch drops the lane's later tuples
        // before their filter loads (8.1 instead of 12.3 per header at 512k rules): the
        // vector-memory data path is busy nearly all of the kernel's time. Batches no
        // lane needs are skipped. (With candidates most lanes enter certification with
        // an answer already, and this variant's 40 VGPRs cost more beside the predictor
        // than its loads save.)
        static_assert(NW == 1, "rank batches use one mask word");
        for (uint32_t r0 = 0; r0 < ntup; r0 += 8) {
            uint32_t want = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t r = r0 + q;
                if (r < ntup && ((todo[0] >> s_order[r]) & 1u) &&
                    kless(s_rank[r].x, s_rank[r].y, b.prio, b.id))
                    want |= 1u << q;
            }
            if (!wave_or(want)) continue;
            if (STATS) ++n_rounds;
            uint32_t wd[8], pos[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                wd[q] = 0;
                pos[q] = 0;
                if ((want >> q) & 1u) {
                    const uint32_t t = s_order[r0 + q];
                    const uint32_t bit =
                        filter_hash(t, sip & s_t[t].smask, dip & s_t[t].dmask) & filter_mask;
                    wd[q] = filter[bit >> 5];
                    pos[q] = bit & 31u;
                    if (STATS) ++n_filter;
                }
            }
            uint32_t pass = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) pass |= ((wd[q] >> pos[q]) & 1u) << q;
            while (pass) {
                const int q = __builtin_ctz(pass);
                pass &= pass - 1u;
                if (STATS) ++steps;
                const uint32_t t = s_order[r0 + q];
                if (!kless(s_t[t].best_prio, s_t[t].best_id, b.prio, b.id)) continue;
                const uint32_t ms = sip & s_t[t].smask, md = dip & s_t[t].dmask;
                search_tuple<STATS>(t, key_hash(t, ms, md), ms, md, sip, dip, sp, dp, proto,
                                    slot_mask, slots, recs, b, n_probe, n_slots, n_recs);
            }
        }
    } else {
    // Phase 1: the filter bits of every remaining tuple, eight tuples per batch with their
    // loads issued back to back; `hits` keeps the tuples whose bit is set. With one mask
    // word a batch is eight consecutive tuples (batches no lane of the wave needs are
    // skipped); with several, each lane takes its own next eight tuples, so the wave runs
    // as many batches as its busiest lane needs rather than one per eight tuple indices.
    uint32_t hits[NW];
    if constexpr (NW > 1) {
        uint32_t rem[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            hits[w] = 0;
            rem[w] = todo[w];
        }
        for (;;) {
            uint32_t left = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) left |= rem[w];
            if (!wave_or(left)) break;  // each batch takes up to eight tuples of every lane
            if (STATS) ++n_rounds;
            uint32_t tq[8], wd[8], pos[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                uint32_t t = kNoTuple;
#pragma unroll
                for (int w = 0; w < NW; ++w)
                    if (t == kNoTuple && rem[w]) {
                        t = 32u * w + (uint32_t)__builtin_ctz(rem[w]);
                        rem[w] &= rem[w] - 1u;
                    }
                tq[q] = t;
                wd[q] = 0;
                pos[q] = 0;
                if (t != kNoTuple) {
                    const uint32_t bit =
                        filter_hash(t, sip & s_t[t].smask, dip & s_t[t].dmask) & filter_mask;
                    wd[q] = filter[bit >> 5];
                    pos[q] = bit & 31u;
                    if (STATS) ++n_filter;
                }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t on = (wd[q] >> pos[q]) & 1u;
#pragma unroll
                for (int w = 0; w < NW; ++w)
                    hits[w] |= ((tq[q] >> 5) == (uint32_t)w ? on : 0u) << (tq[q] & 31u);
            }
        }
    } else {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            hits[w] = 0;
            const uint32_t wave_todo = wave_or(todo[w]);
            if (!wave_todo) continue;
            for (uint32_t t0 = 0; t0 < 32u && 32u * w + t0 < ntup; t0 += 8) {
                if (!((wave_todo >> t0) & 0xFFu)) continue;
                if (STATS) ++n_rounds;
                uint32_t wd[8], pos[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint32_t t = 32u * w + t0 + q;
                    wd[q] = 0;
                    pos[q] = 0;
                    if ((todo[w] >> (t0 + q)) & 1u) {  // t < ntup: todo holds only existing tuples
                        const uint32_t bit =
                            filter_hash(t, sip & s_t[t].smask, dip & s_t[t].dmask) & filter_mask;
                        wd[q] = filter[bit >> 5];
                        pos[q] = bit & 31u;
                        if (STATS) ++n_filter;
                    }
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) hits[w] |= ((wd[q] >> pos[q]) & 1u) << (t0 + q);
            }
        }
    }
    // Phase 2: each lane searches its own passing tuples (so a wave takes as many steps as
    // its busiest lane, not as the union of its lanes' tuples), skipping any whose best key
    // can no longer beat the answer; the order does not matter for the result.
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        while (hits[w]) {
            const uint32_t t = 32u * w + (uint32_t)__builtin_ctz(hits[w]);
            hits[w] &= hits[w] - 1u;
            if (STATS) ++steps;
            if (!kless(s_t[t].best_prio, s_t[t].best_id, b.prio, b.id)) continue;
            const uint32_t ms = sip & s_t[t].smask, md = dip & s_t[t].dmask;
            search_tuple<STATS>(t, key_hash(t, ms, md), ms, md, sip, dip, sp, dp, proto, slot_mask,
                                slots, recs, b, n_probe, n_slots, n_recs);
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
                           size_t n, int kcand, hipStream_t s, bool stats) {
    const size_t chunk = (size_t)1 << 30;
    for (size_t base = 0; base < n; base += chunk) {
        const uint32_t m = (uint32_t)std::min(chunk, n - base);
        const dim3 grid((m + 255) / 256), block(256);
        const uint4* h = reinterpret_cast<const uint4*>(d_hdr) + base;
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, block, 0, s, h, d_out + base, m, rs->d_slots, rs->d_recs,
                               rs->d_cmask, rs->d_filter, rs->d_tt, kcand, rs->d_stats);
        };
        if (rs->nw == 1 && kcand == 0) {
            if (stats) go(k_classify<true, 1, true>);
            else go(k_classify<false, 1, true>);
        } else if (rs->nw == 1) {
            if (stats) go(k_classify<true, 1, false>);
            else go(k_classify<false, 1, false>);
        } else {
            if (stats) go(k_classify<true, kMaskWords, false>);
            else go(k_classify<false, kMaskWords, false>);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tang
