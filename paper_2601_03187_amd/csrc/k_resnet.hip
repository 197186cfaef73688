// The paper's own tuple predictor: the network of Sec. 6.1 with residual blocks (Eq. 1)
// at the size of Sec. 7.1, on the model input of Sec. 6.2:
//   seven 16-bit header chunks / 65535 -> FC(7 -> 512) + ReLU
//   -> n blocks  x <- relu(relu(x w1 + b1) w2 + b2 + x)
//   -> FC(512 -> C) -> top-k (ties to the lower tuple index).
// About 3.2 M multiply-adds per header with 6.3 MB of BF16 weights: the weights cannot
// stay in LDS as the small predictor's do, so every 512 x 512 layer is one MFMA GEMM over
// a chunk of headers. Activations are BF16 rows of 512 per header in a library-owned
// workspace of three chunk buffers (block input / residual, block middle, block output),
// small enough to stay in the Infinity Cache; each layer's 512 KB of weights is read from
// L2 by every workgroup. The input layer (seven inputs) runs in FP32 on the vector ALUs.
//
// MFMA orientation as in the small predictor: weights are the A operand (rows = output
// neurons), headers the B operand (columns). Both operands are read straight from their
// row-major rows: lane group g supplies elements 8g..8g+7 of every 32-wide K block on both
// sides, so the products pair up whatever the instruction's internal K order is. A 16x16
// result leaves lane (g, c) holding neurons 4g..4g+3 of header c: four consecutive BF16 of
// that header's output row, stored as one 8-byte write.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "tang_internal.hpp"

namespace tang {
namespace {

constexpr int kW = 512;               // neurons per layer
constexpr uint32_t kChunk = 65536;    // headers per workspace pass (3 x 64 MB)

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f4 mma(u32x4 a, u32x4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((fl2){a, b}, bf16x2));
}
// ReLU of two packed BF16 as a signed 16-bit max against 0 (RNE keeps signs, so this
// equals rounding after ReLU).
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t p) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, p),
                                                                  (s16x2){0, 0}));
}
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, bytes, 0x00020000);
}

// Input layer: one wave per header, lane l computes neurons 8l..8l+7 (FP32 FMAs over the
// seven chunks, ReLU, BF16) and writes them as one 16-byte store.
__global__ __launch_bounds__(256) void k_res_input(const uint4* __restrict__ hdr, uint32_t m,
                                                   const float* __restrict__ win,
                                                   const float* __restrict__ bin,
                                                   u32x4* __restrict__ x) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    float w[8][7], b[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const uint32_t n = 8u * lane + j;
        b[j] = bin[n];
#pragma unroll
        for (int q = 0; q < 7; ++q) w[j][q] = win[n * 8 + q];
    }
    for (uint32_t p = wave; p < m; p += nwaves) {
        const uint4 h = hdr[p];
        // v / 65535 for a 16-bit v: the FP64 product with 1/65535 rounded to FP32 equals
        // the correctly rounded FP32 quotient for every v (checked exhaustively), at three
        // instructions instead of a full-precision division
        auto seg = [](uint32_t v) { return (float)((double)v * (1.0 / 65535.0)); };
        const float s[7] = {seg(h.x >> 16), seg(h.x & 0xFFFFu), seg(h.y >> 16), seg(h.y & 0xFFFFu),
                            seg(h.z & 0xFFFFu), seg(h.z >> 16), seg(h.w & 0xFFu)};
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            float a = b[j];
#pragma unroll
            for (int q = 0; q < 7; ++q) a = __builtin_fmaf(w[j][q], s[q], a);
            v[j] = a;
        }
        x[(size_t)p * (kW / 8) + lane] =
            (u32x4){relu_bf16x2(pack_bf16(v[0], v[1])), relu_bf16x2(pack_bf16(v[2], v[3])),
                    relu_bf16x2(pack_bf16(v[4], v[5])), relu_bf16x2(pack_bf16(v[6], v[7]))};
    }
}

// One 512 x 512 layer: out = relu(W in + b [+ res]) over m header rows, BF16 in and out,
// FP32 accumulation with the bias as the accumulator's start. Workgroup: 8 waves and 128
// headers; wave w computes neurons 64w..64w+63 (4 row tiles) for all 128 headers (8 column
// tiles). K advances 32 at a time through a ring of three LDS stages, each holding the
// K slice of all 512 weight rows (32 KB) and of the 128 header rows (8 KB). The slices go
// straight from global memory into LDS (global_load_lds, 16 bytes per lane, lane l's
// bytes landing at 16 l from the wave's base), so loads run three steps ahead of the
// MFMAs without holding registers; each wave moves 4 KB of weights and 1 KB of headers
// per step. Rows are 64 bytes with their four 16-byte chunks XOR-swizzled by row bits 1..3
// (chunk c of row n at slot c ^ sw(n), sw(n) = ((n >> 1) ^ (n >> 2)) & 3): any 8, and any
// 16, consecutive rows read at one chunk hit distinct 16-byte bank groups, so 128-bit
// fragment reads are conflict-free whether the LDS serves 8 or 16 lanes per cycle (the
// plain XOR by bits 2..3 left 4 conflict cycles per read). Header rows past m load row m - 1
// instead (their columns are never written). One barrier per step: after it every
// wave's loads for the next step have landed, and nobody still reads the stage that the
// next loads overwrite.
constexpr uint32_t kStageA = 512u * 64u, kStageB = 128u * 64u, kStage = kStageA + kStageB;
__device__ __forceinline__ uint32_t sw(uint32_t row) { return ((row >> 1) ^ (row >> 2)) & 3u; }

template <bool RES>
__global__ __launch_bounds__(512) void k_res_dense(const uint16_t* __restrict__ in,
                                                   const uint16_t* __restrict__ w,
                                                   const float* __restrict__ bias,
                                                   const uint16_t* __restrict__ res,
                                                   uint16_t* __restrict__ out, uint32_t m) {
    __shared__ __attribute__((aligned(16))) unsigned char st0[kStage], st1[kStage], st2[kStage];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, g = lane >> 4, r = lane & 15u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const uint32_t p0 = blockIdx.x * 128u, n0 = wave * 64u;
    // loads: lane l of an instruction fills row 16 j + l / 4 (j: the instruction's row
    // block), slot l % 4, with chunk (l % 4) ^ sw(row); row blocks start at multiples of
    // 16, so sw(row) = sw(l / 4)
    const uint32_t lrow = lane >> 2, lchunk = (lane & 3u) ^ sw(lrow);
    const unsigned char* wsrc = reinterpret_cast<const unsigned char*>(w) +
                                (size_t)(n0 + lrow) * (kW * 2) + lchunk * 16u;
    const uint32_t hrow = std::min(p0 + wave * 16u + lrow, m - 1u);
    const unsigned char* hsrc = reinterpret_cast<const unsigned char*>(in) +
                                (size_t)hrow * (kW * 2) + lchunk * 16u;
    // fragment reads: row (tile base) + r, chunk g at its swizzled slot
    const uint32_t rd = r * 64u + ((g ^ sw(r)) * 16u);
    f4 acc[4][8];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const f4 bv = *reinterpret_cast<const f4*>(bias + n0 + 16 * mt + 4 * g);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt) acc[mt][nt] = bv;
    }
    constexpr int kS = kW / 32;
    auto stage = [&](int k) -> unsigned char* { return k % 3 == 0 ? st0 : k % 3 == 1 ? st1 : st2; };
    auto issue = [&](int kb) {
        unsigned char* sd = stage(kb);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            __builtin_amdgcn_global_load_lds(
                (void*)(wsrc + (size_t)j * 16u * (kW * 2) + kb * 64),
                (__attribute__((address_space(3))) void*)(sd + (wave * 4u + j) * 1024u), 16, 0, 0);
        __builtin_amdgcn_global_load_lds(
            (void*)(hsrc + kb * 64), (__attribute__((address_space(3))) void*)(sd + kStageA + wave * 1024u),
            16, 0, 0);
    };
    // Step hand-off: this wave's LDS reads are done and its loads for the stage read next
    // have landed (s_waitcnt lgkmcnt(0) and vmcnt <= the loads issued since), then a bare
    // barrier. __syncthreads() would add a workgroup release fence, which waits for every
    // load in flight into LDS, the lookahead included; the empty asm statements keep the
    // compiler from moving LDS accesses across the barrier.
    constexpr int kLoadsPerStep = 5;
    auto handoff = [&](int pending) {
        if (pending) __builtin_amdgcn_s_waitcnt(0x0070 | kLoadsPerStep);
        else __builtin_amdgcn_s_waitcnt(0x0070);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
    // Fragments of step k are read from LDS during step k - 1, into the register set
    // k & 1, so their latency hides behind a whole step of MFMAs. Stage k % 3 is refilled
    // (step k + 3) during step k: every wave read it in step k - 1, before that step's
    // closing barrier. Loads of step k + 2 must have landed by the barrier that closes
    // step k, since step k + 1 reads them.
    u32x4 FA[2][4], FB[2][8];
    auto read = [&](int k) {
        const unsigned char* sa = stage(k);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
            FA[k & 1][mt] = *reinterpret_cast<const u32x4*>(sa + (n0 + 16u * mt) * 64u + rd);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
            FB[k & 1][nt] = *reinterpret_cast<const u32x4*>(sa + kStageA + 16u * nt * 64u + rd);
    };
    issue(0);
    issue(1);
    issue(2);
    __builtin_amdgcn_s_waitcnt(0x0070 | (2 * kLoadsPerStep));
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    read(0);
    handoff(1);
#pragma unroll
    for (int kb = 0; kb < kS; ++kb) {
        if (kb + 1 < kS) read(kb + 1);
#pragma unroll
        for (int nt = 0; nt < 8; ++nt)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) acc[mt][nt] = mma(FA[kb & 1][mt], FB[kb & 1][nt], acc[mt][nt]);
        if (kb + 3 < kS) issue(kb + 3);
        if (kb + 2 < kS) handoff(kb + 3 < kS);
    }
#pragma unroll
    for (int nt = 0; nt < 8; ++nt) {
        const uint32_t p = p0 + 16 * nt + r;
        if (p >= m) continue;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const size_t at = (size_t)p * kW + n0 + 16 * mt + 4 * g;
            f4 v = acc[mt][nt];
            if constexpr (RES) {
                const u32x2 xr = *reinterpret_cast<const u32x2*>(res + at);
                v[0] += bf16_lo(xr[0]);
                v[1] += bf16_hi(xr[0]);
                v[2] += bf16_lo(xr[1]);
                v[3] += bf16_hi(xr[1]);
            }
            *reinterpret_cast<u32x2*>(out + at) =
                (u32x2){relu_bf16x2(pack_bf16(v[0], v[1])), relu_bf16x2(pack_bf16(v[2], v[3]))};
        }
    }
}

// Output layer (C scores, no activation) and top-k. Workgroup: 4 waves, each 64 headers
// (4 column tiles); classes in blocks of 32 (2 row tiles), ncb = ceil(C / 32) of them. A
// header's scores of a block sit in the 4 lanes c, c+16, c+32, c+48; each lane keeps a
// running top-4 of the classes it holds (a strictly larger score displaces, so ties keep
// the lower class), which contains the lane's share of any top-k (k <= 4); the top-k is
// then taken across the 4 lanes, ties to the lower class.
__global__ __launch_bounds__(256) void k_res_out(const uint16_t* __restrict__ in,
                                                 const uint16_t* __restrict__ w,
                                                 const float* __restrict__ bias, uint32_t m,
                                                 int C, int topk, uint32_t* __restrict__ cand,
                                                 float* __restrict__ logits,
                                                 uint16_t* __restrict__ cand16) {
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u, g = lane >> 4, r = lane & 15u;
    const uint32_t p0 = (blockIdx.x * 4u + wave) * 64u;
    const int ncb = (C + 31) / 32;
    const __amdgpu_buffer_rsrc_t ri = rsrc(in, m * (uint32_t)(kW * 2));
    const __amdgpu_buffer_rsrc_t rw = rsrc(w, (uint32_t)(32 * ncb * kW * 2));
    const uint32_t boff = (p0 + r) * (kW * 2) + g * 16u;
    float v[4][4];
    int cl[4][4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            v[nt][q] = -INFINITY;
            cl[nt][q] = 1 << 20;
        }
    for (int cb = 0; cb < ncb; ++cb) {
        const uint32_t aoff = (32u * cb + r) * (kW * 2) + g * 16u;
        f4 acc[2][4];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt) {
            const f4 bv = *reinterpret_cast<const f4*>(bias + 32 * cb + 16 * mt + 4 * g);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = bv;
        }
#pragma unroll 2
        for (uint32_t kb = 0; kb < kW / 32; ++kb) {
            u32x4 A[2], B[4];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
                A[mt] = __builtin_amdgcn_raw_buffer_load_b128(rw, aoff, mt * 16 * kW * 2 + kb * 64, 0);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                B[nt] = __builtin_amdgcn_raw_buffer_load_b128(ri, boff, nt * 16 * kW * 2 + kb * 64, 0);
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) acc[mt][nt] = mma(A[mt], B[nt], acc[mt][nt]);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
            const uint32_t pkt = p0 + 16 * nt + r;
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = 32 * cb + 16 * mt + 4 * (int)g + q;
                    const float val = acc[mt][nt][q];
                    if (logits && pkt < m && c < C) logits[(size_t)pkt * C + c] = val;
                    float x = (c < C && val == val) ? val : -INFINITY;
                    int xc = c;
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2) {
                        if (x > v[nt][s2]) {
                            const float tv = v[nt][s2];
                            const int tc = cl[nt][s2];
                            v[nt][s2] = x;
                            cl[nt][s2] = xc;
                            x = tv;
                            xc = tc;
                        }
                    }
                }
        }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const uint32_t pkt = p0 + 16 * nt + r;
        uint32_t packed = 0;
        for (int k = 0; k < topk; ++k) {
            float bv = v[nt][0];
            int bc = cl[nt][0];
#pragma unroll
            for (int q = 1; q < 4; ++q)
                if (v[nt][q] > bv) { bv = v[nt][q]; bc = cl[nt][q]; }
#pragma unroll
            for (int o = 16; o <= 32; o <<= 1) {
                const float ov = __shfl_xor(bv, o, 64);
                const int oc = __shfl_xor(bc, o, 64);
                if (ov > bv || (ov == bv && oc < bc)) { bv = ov; bc = oc; }
            }
            packed |= (uint32_t)bc << (cand_bits(C) * k);
            if (cand16 && g == 0 && pkt < m) cand16[(size_t)pkt * topk + k] = (uint16_t)bc;
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (cl[nt][q] == bc) { v[nt][q] = -INFINITY; cl[nt][q] = 1 << 20; }
        }
        if (cand && g == 0 && pkt < m) cand[pkt] = packed;
    }
}

uint16_t to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

}  // namespace

int resnet_prepare(tang_ruleset_t* rs, const tang_resnet_desc_t* d, const float* const* W,
                   const float* const* b, tang_precision_t p) {
    if (!d || !W || !b) return fail(TANG_EINVAL, "NULL model argument");
    const int C = (int)rs->sigs.size();
    if (d->width != (uint32_t)kW) return fail(TANG_EINVAL, "residual model width must be 512");
    if (d->n_blocks < 1 || d->n_blocks > 16) return fail(TANG_EINVAL, "n_blocks must be in 1..16");
    if ((int)d->n_out != C || C < 1 || C > TANG_MAX_TUPLES)
        return fail(TANG_EINVAL, "output width must equal the number of tuples (1..256)");
    if (d->topk < 1 || (int)d->topk > max_topk(C))
        return fail(TANG_EINVAL, "topk must be in 1..min(4, C), 1..2 above 256 tuples");
    if (p != TANG_BF16) return fail(TANG_EINVAL, "the residual model runs in BF16");
    const int nb = (int)d->n_blocks, L = 2 + 2 * nb;
    for (int l = 0; l < L; ++l)
        if (!W[l] || !b[l]) return fail(TANG_EINVAL, "NULL weight or bias");

    ModelDev m;
    m.kind = 1;
    m.prec = p;
    m.hidden = kW;
    m.n_out = C;
    m.topk = (int)d->topk;
    m.n_blocks = nb;
    std::vector<float> win((size_t)kW * 8, 0.0f);
    for (int n = 0; n < kW; ++n)
        for (int q = 0; q < 7; ++q) win[(size_t)n * 8 + q] = W[0][(size_t)n * 7 + q];
    // biases: input layer, 2 per block, output (classes padded to 32-blocks, zero past C)
    const int CP = kOutPad * ((C + kOutPad - 1) / kOutPad);
    std::vector<float> bias((size_t)(1 + 2 * nb) * kW + CP, 0.0f);
    for (int l = 0; l < 1 + 2 * nb; ++l)
        for (int n = 0; n < kW; ++n) bias[(size_t)l * kW + n] = b[l][n];
    for (int c = 0; c < C; ++c) bias[(size_t)(1 + 2 * nb) * kW + c] = b[L - 1][c];
    // BF16 weights: the block layers [512][512] each, then the output layer [CP][512]
    std::vector<uint16_t> w((size_t)2 * nb * kW * kW + (size_t)CP * kW, 0);
    for (int l = 0; l < 2 * nb; ++l)
        for (size_t k = 0; k < (size_t)kW * kW; ++k) w[(size_t)l * kW * kW + k] = to_bf16(W[1 + l][k]);
    for (int c = 0; c < C; ++c)
        for (int k = 0; k < kW; ++k)
            w[(size_t)2 * nb * kW * kW + (size_t)c * kW + k] = to_bf16(W[L - 1][(size_t)c * kW + k]);

    hipError_t e = dev_alloc(&m.rin, win.size() * 4);
    if (e == hipSuccess) e = hipMemcpy(m.rin, win.data(), win.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = dev_alloc(&m.bias, bias.size() * 4);
    if (e == hipSuccess) e = hipMemcpy(m.bias, bias.data(), bias.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = dev_alloc(&m.rw, w.size() * 2);
    if (e == hipSuccess) e = hipMemcpy(m.rw, w.data(), w.size() * 2, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = dev_alloc(&m.ws, (size_t)3 * kChunk * kW * 2);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&m.ws_done, hipEventDisableTiming);
    if (e != hipSuccess) {
        model_free(m);
        return hip_fail(e, "residual model upload");
    }
    m.bytes = win.size() * 4 + bias.size() * 4 + w.size() * 2 + (size_t)3 * kChunk * kW * 2;
    m.loaded = 1;
    model_free(rs->model);
    rs->model = m;
    rs->version++;
    return TANG_OK;
}

// The workspace is shared by every call on this ruleset: each call's launches wait for
// the previous call's (an event), whatever stream either used.
hipError_t launch_resnet(const tang_ruleset_t* rs, const tang_header_t* d_hdr, size_t n,
                         uint32_t* cand, float* logits, uint16_t* cand16, hipStream_t s) {
    const ModelDev& m = rs->model;
    std::lock_guard<std::mutex> lk(rs->ws_mu);
    hipError_t e = hipSuccess;
    if (m.ws_used) e = hipStreamWaitEvent(s, m.ws_done, 0);
    if (e != hipSuccess) return e;
    const int nb = m.n_blocks;
    const uint16_t* wts = static_cast<const uint16_t*>(m.rw);
    const uint16_t* wout = wts + (size_t)2 * nb * kW * kW;
    const float* bout = m.bias + (size_t)(1 + 2 * nb) * kW;
    for (size_t base = 0; base < n; base += kChunk) {
        const uint32_t c = (uint32_t)std::min<size_t>(kChunk, n - base);
        uint16_t* X = m.ws;
        uint16_t* Hm = X + (size_t)kChunk * kW;
        uint16_t* Y = Hm + (size_t)kChunk * kW;
        const uint32_t gin = std::min<uint32_t>((c + 3) / 4, 2048);
        hipLaunchKernelGGL(k_res_input, dim3(gin), dim3(256), 0, s,
                           reinterpret_cast<const uint4*>(d_hdr + base), c, m.rin, m.bias,
                           reinterpret_cast<u32x4*>(X));
        const dim3 gd((c + 127) / 128);
        for (int k = 0; k < nb; ++k) {
            const uint16_t* w1 = wts + (size_t)(2 * k) * kW * kW;
            const uint16_t* w2 = w1 + (size_t)kW * kW;
            const float* b1 = m.bias + (size_t)(1 + 2 * k) * kW;
            const float* b2 = b1 + kW;
            hipLaunchKernelGGL(k_res_dense<false>, gd, dim3(512), 0, s, X, w1, b1, nullptr, Hm, c);
            hipLaunchKernelGGL(k_res_dense<true>, gd, dim3(512), 0, s, Hm, w2, b2, X, Y, c);
            std::swap(X, Y);
        }
        hipLaunchKernelGGL(k_res_out, dim3((c + 255) / 256), dim3(256), 0, s, X, wout, bout, c,
                           m.n_out, m.topk, cand ? cand + base : nullptr,
                           logits ? logits + base * (size_t)m.n_out : nullptr,
                           cand16 ? cand16 + base * (size_t)m.topk : nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    e = hipEventRecord(m.ws_done, s);
    if (e == hipSuccess) m.ws_used = true;
    return e;
}

}  // namespace tang
