// Build-time and update-time kernels: conflict masks (certification), record moves for
// bucket rewrites, and slot-table scatters.
//
// Conflict mask of rule m: the set of tuples holding a rule r with key(r) < key(m)
// whose 5-field box intersects m's box. If a packet matches m and a better rule r, the
// packet lies in both boxes, so r's tuple is in m's mask; probing those tuples after m
// is found therefore makes the answer exact (the verification the paper leaves to
// future work, Sec. 8). After deletes a mask is a superset, which stays exact.
#include "tang_internal.hpp"

namespace tang {
namespace {

__device__ __forceinline__ bool box_meet(const BoxDev& a, const BoxDev& b) {
    bool ok = (a.slo <= b.shi) & (b.slo <= a.shi) & (a.dlo <= b.dhi) & (b.dlo <= a.dhi);
    ok &= ((a.sp & 0xFFFFu) <= (b.sp >> 16)) & ((b.sp & 0xFFFFu) <= (a.sp >> 16));
    ok &= ((a.dp & 0xFFFFu) <= (b.dp >> 16)) & ((b.dp & 0xFFFFu) <= (a.dp >> 16));
    const uint32_t ea = (a.pt >> 8) & 1u, eb = (b.pt >> 8) & 1u;
    ok &= (ea == 0) | (eb == 0) | ((a.pt & 0xFFu) == (b.pt & 0xFFu));
    return ok;
}

__device__ __forceinline__ BoxDev rec_box(const Rec& r, uint32_t pos) {
    const uint32_t sm = pmask(meta_sl(r.meta)), dm = pmask(meta_dl(r.meta));
    return BoxDev{r.sip, r.sip | ~sm, r.dip, r.dip | ~dm, r.sp, r.dp,
                  meta_proto(r.meta) | (meta_exact(r.meta) << 8) | (meta_tuple(r.meta) << 16), pos};
}

// Mask words of rule at record position p: the record's own word (NW = 1) or a row of
// the side array.
template <int NW>
__device__ __forceinline__ uint32_t* mask_row(Rec* recs, uint32_t* cmask, uint32_t p) {
    if constexpr (NW == 1) return &recs[p].cmask;
    else return cmask + (size_t)p * NW;
}

// One thread per rule i (boxes in ascending key order); rules j < i stream through LDS.
template <int NW>
__global__ __launch_bounds__(256) void k_conflict_build(const BoxDev* __restrict__ boxes,
                                                        uint32_t n, Rec* __restrict__ recs,
                                                        uint32_t* __restrict__ cmask,
                                                        const uint32_t* __restrict__ all_mask) {
    __shared__ BoxDev tile[256];
    const uint32_t base = blockIdx.x * 256u;
    const uint32_t i = base + threadIdx.x;
    const bool valid = i < n;
    BoxDev me = valid ? boxes[i] : BoxDev{0, 0, 0, 0, 0, 0, 0, 0};
    uint32_t mask[NW], full[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        mask[w] = 0;
        full[w] = all_mask[w];
    }
    auto done = [&]() {
        bool f = true;
#pragma unroll
        for (int w = 0; w < NW; ++w) f &= mask[w] == full[w];
        return f;
    };
    const uint32_t j_end = min(n, base + 256u);  // block-uniform
    for (uint32_t j0 = 0; j0 < j_end; j0 += 256u) {
        if (!__syncthreads_or(valid && !done())) break;
        const uint32_t j = j0 + threadIdx.x;
        if (j < n) tile[threadIdx.x] = boxes[j];
        __syncthreads();
        if (valid && !done() && i > j0) {
            const uint32_t cnt = min(256u, i - j0);
            for (uint32_t k = 0; k < cnt; ++k) {
                const uint32_t t = tile[k].pt >> 16;
                const uint32_t tb = 1u << (t & 31u);
                uint32_t& word = mask[NW == 1 ? 0 : t >> 5];
                if (word & tb) continue;
                if (box_meet(me, tile[k])) word |= tb;
            }
        }
        __syncthreads();
    }
    if (valid) {
        uint32_t* row = mask_row<NW>(recs, cmask, me.pos);
#pragma unroll
        for (int w = 0; w < NW; ++w) row[w] = mask[w];
    }
}

// After inserts: every live record p is compared with each fresh rule q. If they meet,
// the better-keyed one's tuple goes into the other's mask.
template <int NW>
__global__ __launch_bounds__(256) void k_conflict_update(Rec* __restrict__ recs,
                                                         uint32_t* __restrict__ cmask, uint32_t used,
                                                         const uint32_t* __restrict__ new_pos,
                                                         uint32_t n_new) {
    __shared__ BoxDev q[256];
    __shared__ uint32_t qkey_p[256], qkey_i[256], qadd[256][NW];
    const uint32_t p = blockIdx.x * 256u + threadIdx.x;
    Rec me;
    bool live = false;
    if (p < used) {
        me = recs[p];
        live = !(me.prio == kDead && me.id == kDead);
    }
    const BoxDev mb = live ? rec_box(me, p) : BoxDev{0, 0, 0, 0, 0, 0, 0, 0};
    const uint32_t my_t = meta_tuple(me.meta);
    uint32_t add[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) add[w] = 0;
    for (uint32_t q0 = 0; q0 < n_new; q0 += 256u) {
        const uint32_t cnt = min(256u, n_new - q0);
        if (threadIdx.x < cnt) {
            const uint32_t pos = new_pos[q0 + threadIdx.x];
            const Rec r = recs[pos];
            q[threadIdx.x] = rec_box(r, pos);
            qkey_p[threadIdx.x] = r.prio;
            qkey_i[threadIdx.x] = r.id;
#pragma unroll
            for (int w = 0; w < NW; ++w) qadd[threadIdx.x][w] = 0;
        }
        __syncthreads();
        if (live) {
            for (uint32_t k = 0; k < cnt; ++k) {
                if (q[k].pos == p || !box_meet(mb, q[k])) continue;
                const bool better = me.prio < qkey_p[k] || (me.prio == qkey_p[k] && me.id < qkey_i[k]);
                if (better) {
                    atomicOr(&qadd[k][NW == 1 ? 0 : my_t >> 5], 1u << (my_t & 31u));
                } else {
                    const uint32_t t = q[k].pt >> 16;
                    add[NW == 1 ? 0 : t >> 5] |= 1u << (t & 31u);
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < cnt) {
            uint32_t* row = mask_row<NW>(recs, cmask, q[threadIdx.x].pos);
#pragma unroll
            for (int w = 0; w < NW; ++w)
                if (qadd[threadIdx.x][w]) atomicOr(&row[w], qadd[threadIdx.x][w]);
        }
        __syncthreads();
    }
    if (live) {
        uint32_t* row = mask_row<NW>(recs, cmask, p);
#pragma unroll
        for (int w = 0; w < NW; ++w)
            if (add[w]) atomicOr(&row[w], add[w]);
    }
}

__global__ void k_stage_records(const Rec* __restrict__ recs, const Rec* __restrict__ fresh,
                                const uint32_t* __restrict__ src, uint32_t n,
                                Rec* __restrict__ stage) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t s = src[i];
    stage[i] = (s & 0x80000000u) ? fresh[s & 0x7FFFFFFFu] : recs[s];
}

__global__ void k_place_records(Rec* __restrict__ recs, const Rec* __restrict__ stage,
                                const uint32_t* __restrict__ dst, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    recs[dst[i]] = stage[i];
}

__global__ void k_stage_masks(const uint32_t* __restrict__ cmask, uint32_t nw,
                              const uint32_t* __restrict__ src, uint32_t n,
                              uint32_t* __restrict__ stage) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * nw) return;
    const uint32_t r = i / nw, w = i % nw, s = src[r];
    stage[i] = (s & 0x80000000u) ? 0u : cmask[(size_t)s * nw + w];
}

__global__ void k_place_masks(uint32_t* __restrict__ cmask, uint32_t nw,
                              const uint32_t* __restrict__ stage, const uint32_t* __restrict__ dst,
                              uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * nw) return;
    cmask[(size_t)dst[i / nw] * nw + i % nw] = stage[i];
}

__global__ void k_scatter_slots(Slot* __restrict__ slots, const uint32_t* __restrict__ idx,
                                const Slot* __restrict__ val, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) slots[idx[i]] = val[i];
}

}  // namespace

hipError_t launch_conflict_build(const BoxDev* d_boxes, size_t n, Rec* d_recs, uint32_t* d_cmask,
                                 uint32_t nw, const uint32_t* all_mask, hipStream_t s) {
    if (!n) return hipSuccess;
    const dim3 g((n + 255) / 256), b(256);
    if (nw == 1)
        hipLaunchKernelGGL(k_conflict_build<1>, g, b, 0, s, d_boxes, (uint32_t)n, d_recs, d_cmask, all_mask);
    else if (nw == kMaskWords)
        hipLaunchKernelGGL(k_conflict_build<kMaskWords>, g, b, 0, s, d_boxes, (uint32_t)n, d_recs,
                           d_cmask, all_mask);
    else
        hipLaunchKernelGGL(k_conflict_build<kMaxWords>, g, b, 0, s, d_boxes, (uint32_t)n, d_recs,
                           d_cmask, all_mask);
    return hipGetLastError();
}

hipError_t launch_conflict_update(Rec* d_recs, uint32_t* d_cmask, uint32_t nw, uint32_t rec_used,
                                  const uint32_t* d_new_pos, uint32_t n_new, hipStream_t s) {
    if (!n_new || !rec_used) return hipSuccess;
    const dim3 g((rec_used + 255) / 256), b(256);
    if (nw == 1)
        hipLaunchKernelGGL(k_conflict_update<1>, g, b, 0, s, d_recs, d_cmask, rec_used, d_new_pos, n_new);
    else if (nw == kMaskWords)
        hipLaunchKernelGGL(k_conflict_update<kMaskWords>, g, b, 0, s, d_recs, d_cmask, rec_used,
                           d_new_pos, n_new);
    else
        hipLaunchKernelGGL(k_conflict_update<kMaxWords>, g, b, 0, s, d_recs, d_cmask, rec_used,
                           d_new_pos, n_new);
    return hipGetLastError();
}

hipError_t launch_move_records(Rec* d_recs, const Rec* d_fresh, const uint32_t* d_src,
                               const uint32_t* d_dst, uint32_t n, Rec* d_stage, hipStream_t s) {
    if (!n) return hipSuccess;
    const dim3 g((n + 255) / 256), b(256);
    hipLaunchKernelGGL(k_stage_records, g, b, 0, s, d_recs, d_fresh, d_src, n, d_stage);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_place_records, g, b, 0, s, d_recs, d_stage, d_dst, n);
    return hipGetLastError();
}

hipError_t launch_move_masks(uint32_t* d_cmask, uint32_t nw, const uint32_t* d_src,
                             const uint32_t* d_dst, uint32_t n, uint32_t* d_stage, hipStream_t s) {
    if (!n) return hipSuccess;
    const dim3 g((n * nw + 255) / 256), b(256);
    hipLaunchKernelGGL(k_stage_masks, g, b, 0, s, d_cmask, nw, d_src, n, d_stage);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_place_masks, g, b, 0, s, d_cmask, nw, d_stage, d_dst, n);
    return hipGetLastError();
}

hipError_t launch_scatter_slots(Slot* d_slots, const uint32_t* d_idx, const Slot* d_val,
                                uint32_t n, hipStream_t s) {
    if (!n) return hipSuccess;
    hipLaunchKernelGGL(k_scatter_slots, dim3((n + 255) / 256), dim3(256), 0, s, d_slots, d_idx,
                       d_val, n);
    return hipGetLastError();
}

}  // namespace tang
