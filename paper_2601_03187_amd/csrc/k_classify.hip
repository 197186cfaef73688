// Search stage of the two-stage classification (Sec. 5.1.1), one packet per lane:
//   1. probe the predicted tuples: truncate SIP/DIP to the tuple's prefix lengths,
//      hash, walk the open-addressing slots to the bucket, and compare the bucket's
//      rules one by one in (priority, id) order -- the first match is the bucket's best;
//   2. certify: if a rule matched, probe the tuples of its conflict mask (the only
//      tuples that can hold a better matching rule); if nothing matched, probe every
//      remaining tuple (the paper's post-verification search, Sec. 5.1.1);
//   in both cases tuples are visited in ascending order of their best key and the
//   search stops once a tuple's best key cannot beat the current answer.
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

template <bool STATS>
__device__ __forceinline__ void probe(uint32_t t, uint32_t sip, uint32_t dip, uint32_t sp,
                                      uint32_t dp, uint32_t proto, const TupleDev* s_t,
                                      uint32_t slot_mask, const Slot* __restrict__ slots,
                                      const Rec* __restrict__ recs, Best& b, uint32_t& n_slots,
                                      uint32_t& n_recs) {
    const uint32_t ms = sip & s_t[t].smask, md = dip & s_t[t].dmask;
    uint32_t h = slot_hash(t, ms, md) & slot_mask;
    // the table is kept at most half full, so an empty slot ends every walk; the step
    // bound only guards against a corrupted table
    for (uint32_t step = 0; step <= slot_mask; ++step) {
        const Slot s = slots[h];
        if (STATS) ++n_slots;
        if (s.tl == kEmptyTL) return;
        if (s.ms == ms && s.md == md && (s.tl >> 24) == t) {
            const uint32_t len = s.tl & kMaxBucketLen;
            for (uint32_t k = 0; k < len; ++k) {
                const Rec r = recs[s.off + k];
                if (STATS) ++n_recs;
                if (!kless(r.prio, r.id, b.prio, b.id)) break;
                if (rec_match(r, sip, dip, sp, dp, proto)) {
                    b = Best{r.prio, r.id, r.cmask, meta_tuple(r.meta)};
                    break;
                }
            }
            return;
        }
        h = (h + 1) & slot_mask;
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
    }
    __syncthreads();
    const uint32_t ntup = s_misc[0], all_mask = s_misc[1], slot_mask = s_misc[2];
    const uint32_t i = blockIdx.x * 256u + tid;
    uint32_t n_probe = 0, n_slots = 0, n_recs = 0, top1 = 0, fb = 0, nm = 0, active = 0;
    if (i < n) {
        active = 1;
        const uint4 h = hdr[i];
        const uint32_t sip = h.x, dip = h.y, sp = h.z & 0xFFFFu, dp = h.z >> 16,
                       proto = h.w & 0xFFu;
        Best b{kDead, kDead, 0u, 0u};
        bool found = false;
        uint32_t probed = 0, c0 = 0xFFu;
        if (kcand > 0) {
            const uint32_t cp = out[i];
            for (int c = 0; c < kcand; ++c) {
                const uint32_t t = (cp >> (8 * c)) & 0xFFu;
                if (c == 0) c0 = t;
                if (t >= ntup || ((probed >> t) & 1u)) continue;
                probed |= 1u << t;
                if (!kless(s_t[t].best_prio, s_t[t].best_id, b.prio, b.id)) continue;
                if (STATS) ++n_probe;
                probe<STATS>(t, sip, dip, sp, dp, proto, s_t, slot_mask, slots, recs, b, n_slots,
                             n_recs);
            }
            found = b.id != kDead || b.prio != kDead;
        }
        uint32_t todo = (found ? b.cmask : all_mask) & ~probed & all_mask;
        if (STATS) fb = found ? 0u : 1u;
        for (uint32_t j = 0; j < ntup && todo; ++j) {
            const uint32_t t = s_order[j];
            if (!((todo >> t) & 1u)) continue;
            if (!kless(s_t[t].best_prio, s_t[t].best_id, b.prio, b.id)) break;
            todo &= ~(1u << t);
            if (STATS) ++n_probe;
            probe<STATS>(t, sip, dip, sp, dp, proto, s_t, slot_mask, slots, recs, b, n_slots, n_recs);
        }
        found = b.id != kDead || b.prio != kDead;
        out[i] = found ? b.id : TANG_NO_MATCH;
        if (STATS) {
            top1 = (found && b.tuple == c0) ? 1u : 0u;
            nm = found ? 0u : 1u;
        }
    }
    if (STATS) {
        unsigned long long v[7] = {active, n_probe, n_slots, n_recs, top1, fb, nm};
#pragma unroll
        for (int q = 0; q < 7; ++q) v[q] = wave_sum(v[q]);
        if ((tid & 63) == 0) {
            atomicAdd(&st->packets, v[0]);
            atomicAdd(&st->probes, v[1]);
            atomicAdd(&st->slots, v[2]);
            atomicAdd(&st->records, v[3]);
            atomicAdd(&st->top1, v[4]);
            atomicAdd(&st->fallbacks, v[5]);
            atomicAdd(&st->nomatch, v[6]);
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
                               rs->d_recs, rs->d_tt, kcand, rs->d_stats);
        else
            hipLaunchKernelGGL(k_classify<false>, grid, block, 0, s, h, d_out + base, m,
                               rs->d_slots, rs->d_recs, rs->d_tt, kcand, rs->d_stats);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tang
