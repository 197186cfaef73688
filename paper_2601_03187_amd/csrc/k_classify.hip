// Search stage of the two-stage classification (Sec. 5.1.1), one packet per lane:
//   1. probe the predicted tuples: truncate SIP/DIP to the tuple's prefix lengths,
//      hash, walk the open-addressing slots to the bucket, and compare the bucket's
//      rules one by one in (priority, id) order -- the first match is the bucket's best;
//   2. certify: if a rule matched, probe the tuples of its conflict mask (the only
//      tuples that can hold a better matching rule); if nothing matched, probe every
//      remaining tuple (the paper's post-verification search, Sec. 5.1.1);
//   in both cases tuples are visited in ascending order of their best key and the
//   search stops once a tuple's best key cannot beat the current answer.
// Before any slot walk, a bit of the bucket filter rules out a tuple that has no bucket
// for the header's masked addresses (most certification probes); the bit is read only for
// tuples the search actually reaches.
// Candidates come packed in the output word (one byte per candidate) from the MLP.
#include "tang_internal.hpp"

namespace tang {
namespace {

struct Best {
    uint32_t prio, id, cmask, tuple;
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

// Compares one list of records in (priority, id) order: the first match is its best;
// the scan stops there or at the first record that cannot beat the current answer.
template <bool STATS>
__device__ __forceinline__ void scan_list(uint32_t off, uint32_t len, uint32_t sip, uint32_t dip,
                                          uint32_t sp, uint32_t dp, uint32_t proto,
                                          const Rec* __restrict__ recs, Best& b, uint32_t& n_recs) {
    for (uint32_t k = 0; k < len; ++k) {
        const Rec r = recs[off + k];
        if (STATS) ++n_recs;
        if (!kless(r.prio, r.id, b.prio, b.id)) break;
        if (rec_match(r, sip, dip, sp, dp, proto)) {
            b = Best{r.prio, r.id, r.cmask, meta_tuple(r.meta)};
            break;
        }
    }
}

// Walks the open-addressing slots to key (tk, k0, k1); returns the slot, or an empty one.
// The table is kept at most a third full, so an empty slot ends every walk; the step
// bound only guards against a corrupted table.
// Walks the open-addressing slots from hash h to key (tk, k0, k1); returns the slot, or
// an empty one. The table is kept at most a third full, so an empty slot ends every
// walk; the step bound only guards against a corrupted table.
template <bool STATS>
__device__ __forceinline__ Slot find_slot(uint64_t h64, uint32_t tk, uint32_t k0, uint32_t k1,
                                          uint32_t slot_mask, const Slot* __restrict__ slots,
                                          uint32_t& n_slots) {
    uint32_t h = slot_of(h64) & slot_mask;
    for (uint32_t step = 0; step <= slot_mask; ++step) {
        const Slot s = slots[h];
        if (STATS) ++n_slots;
        if (s.tl == kEmptyTL || (s.ms == k0 && s.md == k1 && (s.tl >> 24) == tk)) return s;
        h = (h + 1) & slot_mask;
    }
    return Slot{0, 0, kEmptyTL, 0};
}

// Searches tuple t for this header. One hash serves the filter bit (is there a bucket
// for the header's masked key at all?) and the slot walk.
template <bool STATS>
__device__ __forceinline__ void probe(uint32_t t, uint32_t sip, uint32_t dip, uint32_t sp,
                                      uint32_t dp, uint32_t proto, const TupleDev* s_t,
                                      uint32_t slot_mask, uint32_t filter_mask,
                                      const uint32_t* __restrict__ filter,
                                      const Slot* __restrict__ slots, const Rec* __restrict__ recs,
                                      Best& b, uint32_t& n_probe, uint32_t& n_slots,
                                      uint32_t& n_recs) {
    const uint32_t ms = sip & s_t[t].smask, md = dip & s_t[t].dmask;
    const uint64_t h = key_hash(t, ms, md);
    const uint32_t bit = filter_of(h) & filter_mask;
    if (!((filter[bit >> 5] >> (bit & 31u)) & 1u)) return;
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
        const uint32_t tk = t | (keys[q][0] << 5);
        const Slot u = find_slot<STATS>(key_hash(tk, bi, keys[q][1]), tk, bi, keys[q][1], slot_mask,
                                        slots, n_slots);
        if (u.tl != kEmptyTL)
            scan_list<STATS>(u.off, u.tl & kMaxBucketLen, sip, dip, sp, dp, proto, recs, b, n_recs);
    }
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <bool STATS>
__global__ __launch_bounds__(256) void k_classify(const uint4* __restrict__ hdr,
                                                  uint32_t* __restrict__ out, uint32_t n,
                                                  const Slot* __restrict__ slots,
                                                  const Rec* __restrict__ recs,
                                                  const uint32_t* __restrict__ filter,
                                                  const TupleTable* __restrict__ ttg, int kcand,
                                                  StatsDev* __restrict__ st) {
    __shared__ TupleDev s_t[TANG_MAX_TUPLES];
    __shared__ uint32_t s_order[TANG_MAX_TUPLES];
    __shared__ uint32_t s_misc[4];
    const int tid = threadIdx.x;
    if (tid < TANG_MAX_TUPLES) {
        s_t[tid] = ttg->t[tid];
        s_order[tid] = ttg->order[tid];
    }
    if (tid == 0) {
        s_misc[0] = ttg->n;
        s_misc[1] = ttg->all_mask;
        s_misc[2] = ttg->slot_mask;
        s_misc[3] = ttg->filter_mask;
    }
    __syncthreads();
    const uint32_t ntup = s_misc[0], all_mask = s_misc[1], slot_mask = s_misc[2],
                   filter_mask = s_misc[3];
    const uint32_t i = blockIdx.x * 256u + tid;
    uint32_t n_probe = 0, n_slots = 0, n_recs = 0, top1 = 0, fb = 0, nm = 0, active = 0;
    uint32_t sip = 0, dip = 0, sp = 0, dp = 0, proto = 0, todo = 0, c0 = 0xFFu;
    Best b{kDead, kDead, 0u, 0u};
    if (i < n) {
        active = 1;
        const uint4 h = hdr[i];
        sip = h.x;
        dip = h.y;
        sp = h.z & 0xFFFFu;
        dp = h.z >> 16;
        proto = h.w & 0xFFu;
        bool found = false;
        uint32_t probed = 0;
        if (kcand > 0) {
            const uint32_t cp = out[i];
            for (int c = 0; c < kcand; ++c) {
                const uint32_t t = (cp >> (8 * c)) & 0xFFu;
                if (c == 0) c0 = t;
                if (t >= ntup || ((probed >> t) & 1u)) continue;
                probed |= 1u << t;
                if (!kless(s_t[t].best_prio, s_t[t].best_id, b.prio, b.id)) continue;
                probe<STATS>(t, sip, dip, sp, dp, proto, s_t, slot_mask, filter_mask, filter, slots,
                             recs, b, n_probe, n_slots, n_recs);
            }
            found = b.id != kDead;
        }
        todo = (found ? b.cmask : all_mask) & ~probed & all_mask;
        if (STATS) fb = found ? 0u : 1u;
    }
    // The remaining tuples in ascending best-key order. Every lane walks the same order,
    // so the loop, the tuple index and its masks and best key are wave-uniform; a lane
    // probes the tuples of its own list, and drops out once a tuple's best key cannot
    // beat its answer (no later tuple can either).
    for (uint32_t j = 0; j < ntup; ++j) {
        const uint32_t t = __builtin_amdgcn_readfirstlane(s_order[j]);
        const uint32_t bp = __builtin_amdgcn_readfirstlane(s_t[t].best_prio);
        const uint32_t bid = __builtin_amdgcn_readfirstlane(s_t[t].best_id);
        if (todo && !kless(bp, bid, b.prio, b.id)) todo = 0;
        if (!__any(todo != 0)) break;
        if ((todo >> t) & 1u) {
            todo &= ~(1u << t);
            probe<STATS>(t, sip, dip, sp, dp, proto, s_t, slot_mask, filter_mask, filter, slots, recs,
                         b, n_probe, n_slots, n_recs);
        }
    }
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
        __shared__ unsigned long long s_red[4][7];
        unsigned long long v[7] = {active, n_probe, n_slots, n_recs, top1, fb, nm};
#pragma unroll
        for (int q = 0; q < 7; ++q) v[q] = wave_sum(v[q]);
        if ((tid & 63) == 0)
#pragma unroll
            for (int q = 0; q < 7; ++q) s_red[tid >> 6][q] = v[q];
        __syncthreads();
        if (tid < 7) {
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
        if (stats)
            hipLaunchKernelGGL(k_classify<true>, grid, block, 0, s, h, d_out + base, m, rs->d_slots,
                               rs->d_recs, rs->d_filter, rs->d_tt, kcand, rs->d_stats);
        else
            hipLaunchKernelGGL(k_classify<false>, grid, block, 0, s, h, d_out + base, m,
                               rs->d_slots, rs->d_recs, rs->d_filter, rs->d_tt, kcand, rs->d_stats);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tang
