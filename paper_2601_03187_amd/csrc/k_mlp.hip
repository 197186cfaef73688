// Tuple predictor on MFMA: the plain MLP of Sec. 6.1 (FC -> ReLU -> FC -> ReLU -> FC,
// 104 -> H -> H -> C) followed by argmax / top-k over the C tuple scores (Sec. 6.1,
// Sec. 5.1.1), for FP32, BF16 and FP8 (OCP E4M3) operands with FP32 accumulation:
// v_mfma_f32_16x16x4_f32, v_mfma_f32_16x16x32_bf16 and v_mfma_f32_16x16x128_f8f6f4.
//
// Orientation: every layer computes out^T = W * in^T with output neurons as MFMA rows
// (the A operand, weights) and packets as MFMA columns (the B operand, activations).
// A 16x16 MFMA result leaves lane (g = lane/16, c = lane%16) holding rows 4g..4g+3 of
// column c. The next layer's B operand wants, per lane, a few K values of column c; by
// permuting the next layer's weight columns (its K order) once on the host, the rows a
// lane already holds become exactly the K values it must supply, so activations never
// leave registers between layers. Only the A/B symmetry of the MFMA K layout and the
// output layout are relied on, not the hardware's internal K order.
//
// Layer-1 inputs are the header bits (MSB first over SIP, DIP, SP, DP, PROTO), made in
// registers from the 16-byte header: 0/1 are exact in all three formats.
// Weight fragments live in LDS when they fit (160 KB per CU) and are read from global
// (L2-resident) otherwise; biases and the per-layer FP8 scales stay FP32.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <type_traits>

#include "tang_internal.hpp"

namespace tang {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

template <int PREC> struct FragT;
template <> struct FragT<TANG_FP32> { using T = float; static constexpr int KB = 4; };
template <> struct FragT<TANG_BF16> { using T = u32x4; static constexpr int KB = 32; };
template <> struct FragT<TANG_FP8> { using T = u32x8; static constexpr int KB = 128; };

struct MlpArgs {
    int n_out;
    int topk;
    uint32_t n3;      // output-layer fragments stored (2 per K block per 32 classes)
    uint32_t nbias;   // biases stored: 2 H + 32 x class blocks
    float deq[3];
    float inv_a[3];
    // FP8 hidden layers: the requantisation factor into the next layer's input is 2^e;
    // rq = 2^-e is the scaled conversion's operand, rb = 448 * 2^-e the clamp bound in
    // accumulator units
    float rq[2];
    float rb[2];
};

namespace {

__device__ __forceinline__ f4 mma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mma(u32x4 a, u32x4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}
// FP8 (E4M3) x FP8 over a K = 128 block in one instruction (format codes 0 = E4M3 for
// both operands). With both block-scale operands 0 the compiler emits the unscaled
// v_mfma_f32_16x16x128_f8f6f4; the per-layer scales are applied in the epilogues.
__device__ __forceinline__ f4 mma(u32x8 a, u32x8 b, f4 c) {
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(__builtin_bit_cast(i32x8, a),
                                                            __builtin_bit_cast(i32x8, b), c, 0, 0,
                                                            0, 0, 0, 0);
}

__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((fl2){a, b}, bf16x2));
}
// ReLU of two packed BF16 values as one signed 16-bit max against 0: a BF16 with the
// sign bit set is a negative int16, and non-negative BF16 order as their bit patterns.
// RNE rounding never changes a value's sign, so ReLU after the rounding equals rounding
// after ReLU.
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t p) {
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, p),
                                                                  (s16x2){0, 0}));
}
// Four non-negative floats x (already clamped to x 2^e <= 448) -> the four E4M3 bytes of
// x 2^e, RNE, for rq = 2^-e: the scaled conversion divides by the power of two of its
// scale operand, which is exact, so the only rounding is the one onto E4M3.
__device__ __forceinline__ uint32_t pack_fp8(float a, float b, float c, float d, float rq) {
    s16x2 v = {0, 0};
    v = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(v, a, b, rq, false);
    v = __builtin_amdgcn_cvt_scalef32_pk_fp8_f32(v, c, d, rq, true);
    return __builtin_bit_cast(uint32_t, v);
}

// Header words in MSB-first byte order: SIP, DIP, SP:DP, PROTO:0:0:0.
__device__ __forceinline__ uint32_t hword(const uint4& h, int w) {
    return w == 0 ? h.x : w == 1 ? h.y : w == 2 ? ((h.z << 16) | (h.z >> 16)) : ((h.w & 0xFFu) << 24);
}

// B fragment of the input bits for K block kb and lane group g. BF16 and FP8 read it
// from a 256-entry table in LDS indexed by a header byte (one extract and one LDS read
// per byte instead of a chain of per-bit operations); the table entries are made by
// `bits_entry`, the same per-bit rule the FP32 path applies directly.
template <int PREC> struct Bits;
template <> struct Bits<TANG_FP32> {
    // feature f = 4kb + g: byte kb/2, bit (from the MSB) 4(kb&1) + g
    __device__ static __forceinline__ float get(const uint4& h, int kb, int g) {
        const int byte = kb >> 1;
        const uint32_t w = hword(h, byte >> 2);
        const int pos = 8 * (byte & 3) + 4 * (kb & 1) + g;
        return (float)((w >> (31 - pos)) & 1u);
    }
};
template <> struct Bits<TANG_BF16> {
    // features 32kb + 8g + j (j = 0..7): byte 4kb + g, bit (from the MSB) j; a table entry
    // is 4 words, each two BF16 (1.0 = 0x3F80) for bits 2w and 2w + 1 of the byte
    static constexpr int kEntry = 16;
    __device__ static __forceinline__ void entry(uint32_t byte, unsigned char* dst) {
        u32x4 r;
#pragma unroll
        for (int w = 0; w < 4; ++w)
            r[w] = ((byte >> (7 - 2 * w)) & 1u) * 0x3F80u | ((byte >> (6 - 2 * w)) & 1u) * 0x3F800000u;
        *reinterpret_cast<u32x4*>(dst) = r;
    }
    __device__ static __forceinline__ u32x4 get(const uint4& h, int kb, int g, const unsigned char* tab) {
        const uint32_t byte = (hword(h, kb) >> (24 - 8 * g)) & 0xFFu;
        return *reinterpret_cast<const u32x4*>(tab + byte * kEntry);
    }
};
template <> struct Bits<TANG_FP8> {
    // K = 128 in one block: features 32g + j (j = 0..31) are the bits of header word g,
    // most significant first; 1.0 in E4M3 is 0x38. A table entry is the 8 bytes of one
    // header byte's bits (two words of the fragment).
    static constexpr int kEntry = 8;
    __device__ static __forceinline__ void entry(uint32_t byte, unsigned char* dst) {
        u32x2 r;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            uint32_t v = 0;
#pragma unroll
            for (int b = 0; b < 4; ++b) v |= ((byte >> (7 - 4 * half - b)) & 1u) * (0x38u << (8 * b));
            r[half] = v;
        }
        *reinterpret_cast<u32x2*>(dst) = r;
    }
    __device__ static __forceinline__ u32x8 get(const uint4& h, int, int g, const unsigned char* tab) {
        const uint32_t w = g == 0 ? h.x : g == 1 ? h.y : g == 2 ? ((h.z << 16) | (h.z >> 16))
                                                                : ((h.w & 0xFFu) << 24);
        u32x8 r;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const u32x2 e = *reinterpret_cast<const u32x2*>(tab + ((w >> (24 - 8 * k)) & 0xFFu) * kEntry);
            r[2 * k] = e[0];
            r[2 * k + 1] = e[1];
        }
        return r;
    }
};

// One lane's A fragment `frag` of a layer: from LDS, or from global memory through a
// buffer descriptor (lane offset in one VGPR, fragment offset as a scalar; reads past the
// layer's size return zero instead of faulting). A fragment is stored as 64 consecutive
// lane slots of at most 16 bytes; the 32-byte FP8 fragment as two such planes (bytes
// 0-15 of every lane, then bytes 16-31), so that 128-bit LDS reads stay free of bank
// conflicts.
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, float*) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
}
__device__ __forceinline__ u32x2 bload(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, u32x2*) {
    return __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0);
}
__device__ __forceinline__ u32x4 bload(__amdgpu_buffer_rsrc_t r, uint32_t v, uint32_t s, u32x4*) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, v, s, 0);
}

//
// An LDS read takes one address register plus an immediate offset below 64 KB. Each
// layer's fragments are therefore addressed through 64 KB windows: `win[w]` holds w as
// a value the compiler cannot see (set once per tile), so the window's base becomes one
// register per window instead of one address addition per fragment read past 64 KB.
template <bool IN_LDS, typename F>
__device__ __forceinline__ F ldf(const F* lds, __amdgpu_buffer_rsrc_t r, uint32_t frag, uint32_t lane,
                                 uint32_t sbase, const uint32_t* win) {
    constexpr uint32_t FPW = 65536u / (64u * (uint32_t)sizeof(F));   // fragments per window
    if constexpr (sizeof(F) == 32) {
        u32x4 lo, hi;
        if constexpr (IN_LDS) {
            const u32x4* p = reinterpret_cast<const u32x4*>(reinterpret_cast<const char*>(lds) +
                                                            win[frag / FPW] * 65536u) + lane;
            lo = p[(frag % FPW) * 128];
            hi = p[(frag % FPW) * 128 + 64];
        } else {
            lo = __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16u + sbase, frag * 2048u, 0);
            hi = __builtin_amdgcn_raw_buffer_load_b128(r, lane * 16u + sbase, frag * 2048u + 1024u, 0);
        }
        return (F){lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    } else {
        if constexpr (IN_LDS)
            return reinterpret_cast<const F*>(reinterpret_cast<const char*>(lds) +
                                              win[frag / FPW] * 65536u)[(frag % FPW) * 64 + lane];
        else return bload(r, lane * (uint32_t)sizeof(F) + sbase, frag * 64u * (uint32_t)sizeof(F), (F*)nullptr);
    }
}

// Accumulator start of one 16-row output tile: hidden layers fold the bias in as the
// MFMA's C operand (the four rows this lane holds; FP8 biases are stored in accumulator
// units, b / (s_a s_w)).
template <int PREC>
__device__ __forceinline__ f4 acc_init(const float* sbias, int mt, int g) {
    return *reinterpret_cast<const f4*>(sbias + 16 * mt + 4 * g);
}

// ReLU of one 16-row output tile and conversion into the next layer's B operand. FP8:
// the next input is E4M3(2^e relu(acc)) clamped to 448: one median-of-three against
// [0, rb = 448 2^-e] and the scaled conversion by rq = 2^-e (two values per instruction).
template <int PREC, int NT, int KBN>
__device__ __forceinline__ void epi_hidden(const f4 (&acc)[NT], int mt, float rq, float rb,
                                           typename FragT<PREC>::T (&dst)[KBN][NT]) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
        if constexpr (PREC == TANG_FP32) {
#pragma unroll
            for (int r = 0; r < 4; ++r) dst[4 * mt + r][nt] = fmaxf(acc[nt][r], 0.0f);
        } else if constexpr (PREC == TANG_BF16) {
            dst[mt >> 1][nt][2 * (mt & 1)] = relu_bf16x2(pack_bf16(acc[nt][0], acc[nt][1]));
            dst[mt >> 1][nt][2 * (mt & 1) + 1] = relu_bf16x2(pack_bf16(acc[nt][2], acc[nt][3]));
        } else {
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = __builtin_amdgcn_fmed3f(acc[nt][r], 0.0f, rb);
            // a 128-wide K block holds the rows of 8 consecutive output tiles
            dst[mt >> 3][nt][mt & 7] = pack_fp8(v[0], v[1], v[2], v[3], rq);
        }
    }
}

constexpr int kNoClass = 1 << 20;  // an empty or removed top-k slot (above every class)

// OUTB: most blocks of 32 output classes (1, or 16 for up to 512 tuples; the W3 fragments
// of a multi-block model are read from L2).
template <int PREC, int H, int NT, int LDSM, int WAVES, int OUTB>
__global__ __launch_bounds__(64 * WAVES) void k_mlp(
    const uint4* __restrict__ hdr, uint32_t n, const typename FragT<PREC>::T* __restrict__ w1,
    const typename FragT<PREC>::T* __restrict__ w2, const typename FragT<PREC>::T* __restrict__ w3,
    const u32x4* __restrict__ w1x3, const float* __restrict__ bias_g, MlpArgs a, uint32_t* __restrict__ cand,
    float* __restrict__ logits, uint16_t* __restrict__ cand16, const uint32_t* __restrict__ live) {
    using F = typename FragT<PREC>::T;
    constexpr int KB = FragT<PREC>::KB;
    constexpr int KBN1 = kInPad / KB, KBNH = H / KB, MTH = H / 16;
    // FP32 input blocks past feature 104 are all-zero on both operands: skipped
    constexpr int KBN1_USED = PREC == TANG_FP32 ? 104 / KB : KBN1;
    constexpr uint32_t n1 = MTH * KBN1 * 64, n2 = MTH * KBNH * 64, n3 = 2 * KBNH * 64;
    static_assert(OUTB == 1 || !(LDSM & 4), "multi-block output layers stay in L2");
    // output tiles per MFMA group in layer 2 (more when each tile is only 1-2 MFMAs)
    constexpr int TG = PREC == TANG_FP8 ? 2 : PREC == TANG_BF16 ? 2 : 1;

    if (live) n = min(n, *live);
    // a workgroup without a tile leaves before staging the weights (uniform over the block)
    if (blockIdx.x * WAVES >= (n + 16 * NT - 1) / (16 * NT)) return;

    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    F* s1 = reinterpret_cast<F*>(smem);
    F* s2 = s1 + ((LDSM & 1) ? n1 : 0);
    F* s3 = s2 + ((LDSM & 2) ? n2 : 0);
    float* sb = reinterpret_cast<float*>(s3 + ((LDSM & 4) ? n3 : 0));
    unsigned char* stab = reinterpret_cast<unsigned char*>(sb + 2 * H + kOutPad * OUTB);  // bit table

    {   // stage resident weights and the biases
        auto copy16 = [&](void* dst, const void* src, uint32_t bytes) {
            uint4* d = reinterpret_cast<uint4*>(dst);
            const uint4* s = reinterpret_cast<const uint4*>(src);
            for (uint32_t k = threadIdx.x; k < bytes / 16; k += blockDim.x) d[k] = s[k];
        };
        if (LDSM & 1) copy16(s1, w1, n1 * sizeof(F));
        if (LDSM & 2) copy16(s2, w2, n2 * sizeof(F));
        if (LDSM & 4) copy16(s3, w3, n3 * sizeof(F));
        copy16(sb, bias_g, a.nbias * sizeof(float));
        // FP32 runs its input layer on BF16 MFMAs, so it builds the BF16 bit table
        using BT = Bits<PREC == TANG_FP32 ? TANG_BF16 : PREC>;
        if (threadIdx.x < 256) BT::entry(threadIdx.x, stab + threadIdx.x * BT::kEntry);
    }
    __syncthreads();

    const __amdgpu_buffer_rsrc_t r1 = __builtin_amdgcn_make_buffer_rsrc((void*)w1, 0, n1 * sizeof(F), 0x00020000);
    const __amdgpu_buffer_rsrc_t r2 = __builtin_amdgcn_make_buffer_rsrc((void*)w2, 0, n2 * sizeof(F), 0x00020000);
    const __amdgpu_buffer_rsrc_t r3 = __builtin_amdgcn_make_buffer_rsrc((void*)w3, 0, a.n3 * sizeof(F), 0x00020000);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, col = lane & 15;
    const uint32_t tiles = (n + 16 * NT - 1) / (16 * NT);
    const int C = a.n_out;
    for (uint32_t tile = blockIdx.x * WAVES + wave; tile < tiles; tile += gridDim.x * WAVES) {
        const uint32_t pbase = tile * 16u * NT;
        // the weight loads (LDS and global) are loop-invariant; an opaque zero in their
        // addresses hides that from LICM, which would otherwise hoist every fragment out
        // of the tile loop and run out of registers
        uint32_t sbase = 0;
        asm volatile("" : "+s"(sbase));
        uint32_t win[3] = {0u, 1u, 2u};   // LDS windows (see ldf); 160 KB of LDS needs three
        asm volatile("" : "+v"(win[0]), "+v"(win[1]), "+v"(win[2]));
        // biases and the bit table sit past 64 KB too: their reads go through an opaque
        // base register as well
        const float* sbv = reinterpret_cast<const float*>(reinterpret_cast<const char*>(sb) + win[0] * 65536u);
        const unsigned char* stv = stab + win[0] * 65536u;
        uint4 hv[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const uint32_t p = pbase + nt * 16 + col;
            hv[nt] = p < n ? hdr[p] : make_uint4(0, 0, 0, 0);
        }
        // layer 1: bits -> H.
        F a0[KBNH][NT];
        if constexpr (PREC == TANG_FP32) {
            // FP32 weights against 0/1 inputs: W1 = hi + mid + lo, three BF16 planes that
            // sum to it exactly, so each product with a bit is exact on a BF16 MFMA and
            // the 16x16x32 instruction does 32 of them where 16x16x4 FP32 does 4; the
            // accumulation stays FP32. Fragments (mt, kb, plane) come from L2; the other
            // waves' layer-2 MFMAs cover their latency.
            u32x4 xb[4][NT];
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) xb[kb][nt] = Bits<TANG_BF16>::get(hv[nt], kb, g, stv);
            const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
                (void*)w1x3, 0, (uint32_t)(MTH * 12 * 64 * 16), 0x00020000);
#pragma unroll
            for (int mt = 0; mt < MTH; ++mt) {
                u32x4 wf[12];
#pragma unroll
                for (int f = 0; f < 12; ++f)
                    wf[f] = bload(rx, lane * 16u + sbase, (uint32_t)((mt * 12 + f) * 1024), (u32x4*)nullptr);
                f4 acc[NT];
                const f4 b0 = acc_init<PREC>(sbv, mt, g);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[nt] = b0;
#pragma unroll
                for (int f = 0; f < 12; ++f)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) acc[nt] = mma(wf[f], xb[f / 3][nt], acc[nt]);
                epi_hidden<PREC, NT, KBNH>(acc, mt, a.rq[0], a.rb[0], a0);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
        // When its fragments come from L2 (not LDS), the next tile's
        // loads are issued before this tile's MFMAs so their latency is hidden.
        F pre[KBN1_USED];
        // BF16 / FP8: the input-bit fragments are built once per tile of headers
        F bits[KBN1_USED][NT];
#pragma unroll
        for (int kb = 0; kb < KBN1_USED; ++kb)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bits[kb][nt] = Bits<PREC>::get(hv[nt], kb, g, stv);
        if constexpr (!(LDSM & 1)) {
#pragma unroll
            for (int kb = 0; kb < KBN1_USED; ++kb) pre[kb] = ldf<false>(s1, r1, kb, lane, sbase, win);
        }
#pragma unroll
        for (int mt = 0; mt < MTH; ++mt) {
            F cur[KBN1_USED];
#pragma unroll
            for (int kb = 0; kb < KBN1_USED; ++kb) {
                if constexpr ((LDSM & 1) != 0) cur[kb] = ldf<true>(s1, r1, mt * KBN1 + kb, lane, sbase, win);
                else cur[kb] = pre[kb];
            }
            if constexpr (!(LDSM & 1)) {
                if (mt + 1 < MTH) {
#pragma unroll
                    for (int kb = 0; kb < KBN1_USED; ++kb)
                        pre[kb] = ldf<false>(s1, r1, (mt + 1) * KBN1 + kb, lane, sbase, win);
                }
            }
            f4 acc[NT];
            const f4 b0 = acc_init<PREC>(sbv, mt, g);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[nt] = b0;
#pragma unroll
            for (int kb = 0; kb < KBN1_USED; ++kb) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[nt] = mma(cur[kb], bits[kb][nt], acc[nt]);
            }
            epi_hidden<PREC, NT, KBNH>(acc, mt, a.rq[0], a.rb[0], a0);
            // keep the scheduler from hoisting every tile's fragment loads (register blow-up)
            __builtin_amdgcn_sched_barrier(0);
        }
        }
        // layer 2: H -> H, TG output tiles per group: all MFMAs of the group are issued
        // before its epilogues, so the matrix pipe has independent work while results land.
        // With one block of classes the output layer runs inside this loop: as soon as
        // the group completes a K block of layer 3, that block's MFMAs are issued, so the
        // second hidden layer never has to be held whole (its K blocks are consumed in
        // the same ascending order as an unfused layer 3 would take them).
        F a1[KBNH][NT];
        f4 z[2][NT];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) z[mt][nt] = (f4){0, 0, 0, 0};
        auto layer3_block = [&](int kb) {
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const F A = ldf<(LDSM & 4) != 0>(s3, r3, mt * KBNH + kb, lane, sbase, win);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) z[mt][nt] = mma(A, a1[kb][nt], z[mt][nt]);
            }
        };
#pragma unroll
        for (int mt0 = 0; mt0 < MTH; mt0 += TG) {
            f4 acc[TG][NT];
#pragma unroll
            for (int u = 0; u < TG; ++u) {
                const f4 b0 = acc_init<PREC>(sbv + H, mt0 + u, g);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[u][nt] = b0;
            }
#pragma unroll
            for (int kb = 0; kb < KBNH; ++kb) {
#pragma unroll
                for (int u = 0; u < TG; ++u) {
                    const F A = ldf<(LDSM & 2) != 0>(s2, r2, (mt0 + u) * KBNH + kb, lane, sbase, win);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) acc[u][nt] = mma(A, a0[kb][nt], acc[u][nt]);
                }
            }
#pragma unroll
            for (int u = 0; u < TG; ++u)
                epi_hidden<PREC, NT, KBNH>(acc[u], mt0 + u, a.rq[1], a.rb[1], a1);
            if constexpr (OUTB == 1) {
                // output tile mt feeds K block mt / (KB / 16) (KB >= 16), or the four
                // blocks 4 mt .. 4 mt + 3 (FP32, KB = 4)
#pragma unroll
                for (int u = 0; u < TG; ++u) {
                    const int mt = mt0 + u;
                    if constexpr (KB >= 16) {
                        if ((mt + 1) % (KB / 16) == 0) layer3_block(mt / (KB / 16));
                    } else {
#pragma unroll
                        for (int q = 0; q < 16 / KB; ++q) layer3_block((16 / KB) * mt + q);
                    }
                }
            }
            // FP8 groups are left to the scheduler, which then overlaps one group's scale /
            // clamp / conversion epilogue with the next group's MFMAs (chunked classify
            // 3.17 -> 3.07 ms per 16M headers); for BF16 the same freedom was slower
            // (predictor 2.48 -> 2.60 ms)
            if constexpr (PREC != TANG_FP8) __builtin_amdgcn_sched_barrier(0);
        }
        // layer 3: H -> C in blocks of 32 classes (two 16-row tiles). With one block each
        // lane's 8 scores go straight to the top-k; with more, each lane keeps a running
        // top-k of the classes it holds (a strictly larger score displaces, so ties keep
        // the lower class, as classes ascend block by block; there a NaN or -inf score
        // counts as -FLT_MAX, so every real class beats an empty slot and a padded class).
        // With one block a NaN score counts as -inf and ties go to the lower class.
        const float* sb3 = sbv + 2 * H;
        constexpr int KL = OUTB == 1 ? 8 : 4;
        float v[NT][KL];
        int cl[NT][KL];
        if constexpr (OUTB > 1) {
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int q = 0; q < KL; ++q) {
                    v[nt][q] = -INFINITY;
                    cl[nt][q] = kNoClass;
                }
        }
        const int ncb = OUTB == 1 ? 1 : (C + 31) / 32;
#pragma unroll 1
        for (int cb = 0; cb < ncb; ++cb) {
            if constexpr (OUTB > 1) {
#pragma unroll
                for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) z[mt][nt] = (f4){0, 0, 0, 0};
#pragma unroll
                    for (int kb = 0; kb < KBNH; ++kb) {
                        const F A = ldf<(LDSM & 4) != 0>(s3, r3, (2 * cb + mt) * KBNH + kb, lane, sbase, win);
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt) z[mt][nt] = mma(A, a1[kb][nt], z[mt][nt]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // scores; the running top-k keeps topk slots (1, 2, or 4 for 3 and 4; a uniform
            // branch per block picks the count)
            auto scores = [&](auto slots) {
                constexpr int KS = decltype(slots)::value;
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const uint32_t pkt = pbase + nt * 16 + col;
#pragma unroll
                    for (int mt = 0; mt < 2; ++mt) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int c = 32 * cb + 16 * mt + 4 * g + r;
                            float val = (PREC == TANG_FP8 ? z[mt][nt][r] * a.deq[2] : z[mt][nt][r]) + sb3[c];
                            if (logits && pkt < n && c < C) logits[(size_t)pkt * C + c] = val;
                            if constexpr (OUTB == 1) {
                                v[nt][4 * mt + r] = (c < C && val == val) ? val : -INFINITY;
                                cl[nt][4 * mt + r] = c;
                            } else {
                                float x = c < C ? (val == val ? fmaxf(val, -FLT_MAX) : -FLT_MAX) : -INFINITY;
                                int xc = c;
#pragma unroll
                                for (int q = 0; q < KS; ++q) {
                                    if (x > v[nt][q]) {
                                        const float tv = v[nt][q];
                                        const int tc = cl[nt][q];
                                        v[nt][q] = x;
                                        cl[nt][q] = xc;
                                        x = tv;
                                        xc = tc;
                                    }
                                }
                            }
                        }
                    }
                }
            };
            if (OUTB > 1 && a.topk == 1) scores(std::integral_constant<int, 1>{});
            else if (OUTB > 1 && a.topk == 2) scores(std::integral_constant<int, 2>{});
            else scores(std::integral_constant<int, KL>{});
        }
        // top-k with ties to the lower tuple index
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const uint32_t pkt = pbase + nt * 16 + col;
            uint32_t packed = 0;
            for (int k = 0; k < a.topk; ++k) {
                float bv = v[nt][0];
                int bc = cl[nt][0];
#pragma unroll
                for (int q = 1; q < KL; ++q)
                    if (v[nt][q] > bv) { bv = v[nt][q]; bc = cl[nt][q]; }   // lower classes first
#pragma unroll
                for (int o = 16; o <= 32; o <<= 1) {
                    const float ov = __shfl_xor(bv, o, 64);
                    const int oc = __shfl_xor(bc, o, 64);
                    if (ov > bv || (ov == bv && oc < bc)) { bv = ov; bc = oc; }
                }
                packed |= (uint32_t)bc << (cand_bits(C) * k);
                if (cand16 && g == 0 && pkt < n) cand16[(size_t)pkt * a.topk + k] = (uint16_t)bc;
#pragma unroll
                for (int q = 0; q < KL; ++q)
                    if (cl[nt][q] == bc) v[nt][q] = -INFINITY;
                // a removed class must never win again: push it below -inf ties
#pragma unroll
                for (int q = 0; q < KL; ++q)
                    if (cl[nt][q] == bc) cl[nt][q] = kNoClass;
            }
            if (cand && g == 0 && pkt < n) cand[pkt] = packed;
        }
    }
}

// ---------------------------------------------------------------------------------------
// Host side: quantisers, fragment swizzle, upload, launch.

uint16_t f32_to_bf16(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// OCP FP8 E4M3: bias 7, 3 fraction bits, no infinity, max 448; RNE, saturating.
uint8_t f32_to_e4m3(float f) {
    const uint8_t sign = std::signbit(f) ? 0x80 : 0x00;
    double x = std::fabs((double)f);
    if (x != x) return 0x7F;
    if (x >= 448.0) return sign | 0x7E;
    if (x < std::ldexp(1.0, -6)) return sign | (uint8_t)std::nearbyint(x * 512.0);
    int e;
    const double m = std::frexp(x, &e);  // x = m 2^e, m in [0.5, 1)
    int E = e - 1;
    double f8 = std::nearbyint((2.0 * m - 1.0) * 8.0);
    if (f8 == 8.0) { ++E; f8 = 0.0; }
    int code = ((E + 7) << 3) | (int)f8;
    if (code > 0x7E) code = 0x7E;
    return sign | (uint8_t)code;
}

// Input column (of W[out][in]) that lane group g, element j of K block kb carries.
int in_col(int prec, int layer, int kb, int g, int j) {
    if (prec == TANG_FP32) return layer == 0 ? 4 * kb + g : 16 * (kb / 4) + 4 * g + (kb % 4);
    if (prec == TANG_BF16)
        return layer == 0 ? 32 * kb + 8 * g + j : 16 * (2 * kb + (j >> 2)) + 4 * g + (j & 3);
    return layer == 0 ? 128 * kb + 32 * g + j : 16 * (8 * kb + (j >> 2)) + 4 * g + (j & 3);
}

}  // namespace

void model_free(ModelDev& m) {
    for (auto& p : m.w) {
        if (p) dev_release(p);
        p = nullptr;
    }
    if (m.bias) dev_release(m.bias);
    m.bias = nullptr;
    if (m.w1x3) dev_release(m.w1x3);
    m.w1x3 = nullptr;
    if (m.rin) dev_release(m.rin);
    if (m.rw) dev_release(m.rw);
    if (m.ws) dev_release(m.ws);
    if (m.ws_done) hipEventDestroy(m.ws_done);
    m.rin = nullptr;
    m.rw = nullptr;
    m.ws = nullptr;
    m.ws_done = nullptr;
    m.ws_used = false;
    m.kind = 0;
    m.loaded = 0;
    m.bytes = 0;
}

int model_prepare(tang_ruleset_t* rs, const tang_mlp_desc_t* d, const float* const* W,
                  const float* const* b, tang_precision_t p, const float* act_scales) {
    if (!d || !W || !b) return fail(TANG_EINVAL, "NULL model argument");
    const int C = (int)rs->sigs.size();
    if (d->n_layers != 3) return fail(TANG_EINVAL, "only 3-layer MLPs (104 -> H -> H -> C) are supported");
    if (d->dims[0] != 104) return fail(TANG_EINVAL, "input width must be 104 header bits");
    const int H = (int)d->dims[1];
    if ((int)d->dims[2] != H || (H != 128 && H != 256))
        return fail(TANG_EINVAL, "hidden widths must be equal and 128 or 256");
    if ((int)d->dims[3] != C || C < 1 || C > TANG_MAX_TUPLES)
        return fail(TANG_EINVAL, "output width must equal the number of tuples");
    if (d->topk < 1 || (int)d->topk > max_topk(C))
        return fail(TANG_EINVAL, "topk must be in 1..min(4, C), 1..2 above 256 tuples");
    if (p != TANG_FP32 && p != TANG_BF16 && p != TANG_FP8) return fail(TANG_EINVAL, "bad precision");
    if (p == TANG_FP8) {
        if (!act_scales) return fail(TANG_EINVAL, "FP8 needs act_scales");
        for (int l = 1; l < 3; ++l)
            if (!(act_scales[l] > 0.0f) || !std::isfinite(act_scales[l]))
                return fail(TANG_EINVAL, "act_scales must be positive and finite");
    } else if (act_scales) {
        return fail(TANG_EINVAL, "act_scales only apply to FP8");
    }
    for (int l = 0; l < 3; ++l)
        if (!W[l] || !b[l]) return fail(TANG_EINVAL, "NULL weight or bias");

    ModelDev m;
    m.prec = p;
    m.hidden = H;
    m.n_out = C;
    m.topk = (int)d->topk;
    const int KB = p == TANG_FP32 ? 4 : p == TANG_BF16 ? 32 : 128;
    const int E = p == TANG_FP32 ? 1 : p == TANG_BF16 ? 8 : 32;
    const int esz = p == TANG_FP32 ? 4 : p == TANG_BF16 ? 2 : 1;
    const int CP = kOutPad * ((C + kOutPad - 1) / kOutPad);  // classes padded to 32-blocks
    const int outs[3] = {H, H, C}, ins[3] = {104, H, H};
    const int outp[3] = {H, H, CP}, inp[3] = {kInPad, H, H};
    m.w3frags = (uint32_t)(CP / 16 * (H / KB) * 64);
    for (int l = 0; l < 3; ++l) {
        float s_w = 1.0f, inv_w = 1.0f, s_a = 1.0f;
        if (p == TANG_FP8) {
            float amax = 0.0f;
            for (size_t k = 0; k < (size_t)outs[l] * ins[l]; ++k) amax = std::max(amax, std::fabs(W[l][k]));
            s_w = amax > 0.0f ? amax / 448.0f : 1.0f;
            s_a = l == 0 ? 1.0f : act_scales[l];
            if (l < 2) {
                // hidden layer: the weight scale is raised by a factor in [1, 2) until the
                // requantisation factor s_w s_a / s_next is a power of two, 2^e
                const double s_n = act_scales[l + 1];
                int ex = 0;
                const double mant = std::frexp((double)s_w * (double)s_a / s_n, &ex);
                const int e = mant == 0.5 ? ex - 1 : ex;
                if (e < -100 || e > 100) return fail(TANG_EINVAL, "FP8 scales too far apart (|e| > 100)");
                s_w = (float)std::ldexp(s_n / (double)s_a, e);
                m.rq[l] = std::ldexp(1.0f, -e);
            }
            inv_w = 1.0f / s_w;
            m.deq[l] = s_a * s_w;
            m.inv_a[l] = 1.0f / s_a;
        }
        const int MT = outp[l] / 16, KBN = inp[l] / KB;
        std::vector<unsigned char> buf((size_t)MT * KBN * 64 * E * esz, 0);
        for (int mt = 0; mt < MT; ++mt)
            for (int kb = 0; kb < KBN; ++kb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < E; ++j) {
                        const int row = 16 * mt + (lane & 15), g = lane >> 4;
                        const int c = in_col(p, l, kb, g, j);
                        const float w = (row < outs[l] && c < ins[l]) ? W[l][(size_t)row * ins[l] + c] : 0.0f;
                        // FP8: two 16-byte planes per fragment (bytes j < 16, then j >= 16)
                        const size_t frag = (size_t)mt * KBN + kb;
                        const size_t at = p == TANG_FP8
                                              ? ((frag * 2 + j / 16) * 64 + lane) * 16 + j % 16
                                              : ((frag * 64 + lane) * E + j) * esz;
                        if (p == TANG_FP32) std::memcpy(&buf[at], &w, 4);
                        else if (p == TANG_BF16) {
                            const uint16_t q = f32_to_bf16(w);
                            std::memcpy(&buf[at], &q, 2);
                        } else {
                            buf[at] = f32_to_e4m3(w * inv_w);
                        }
                    }
        hipError_t e = dev_alloc(&m.w[l], buf.size());
        if (e == hipSuccess) e = hipMemcpy(m.w[l], buf.data(), buf.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) { model_free(m); return hip_fail(e, "model upload"); }
        m.wbytes[l] = buf.size();
        m.bytes += buf.size();
    }
    if (p == TANG_FP32) {
        // W1 as three BF16 planes in BF16 layer-0 fragment order: hi = w cut to BF16
        // (low 16 bits dropped), mid = (w - hi) cut likewise, lo = w - hi - mid. Each
        // difference is exact in FP32 and lo keeps at most 8 significant bits, so
        // hi + mid + lo = w exactly; cutting (not rounding) never overflows to infinity.
        const int MT = H / 16;
        std::vector<uint16_t> x3((size_t)MT * 4 * 3 * 64 * 8, 0);
        for (int mt = 0; mt < MT; ++mt)
            for (int kb = 0; kb < 4; ++kb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < 8; ++j) {
                        const int row = 16 * mt + (lane & 15), c = in_col(TANG_BF16, 0, kb, lane >> 4, j);
                        const float w = c < 104 ? W[0][(size_t)row * 104 + c] : 0.0f;
                        uint16_t q[3];
                        float rest = w;
                        for (int pl = 0; pl < 3; ++pl) {
                            uint32_t u;
                            std::memcpy(&u, &rest, 4);
                            q[pl] = (uint16_t)(u >> 16);
                            u &= 0xFFFF0000u;
                            float back;
                            std::memcpy(&back, &u, 4);
                            rest -= back;
                        }
                        for (int pl = 0; pl < 3; ++pl)
                            x3[((((size_t)mt * 4 + kb) * 3 + pl) * 64 + lane) * 8 + j] = q[pl];
                    }
        hipError_t e = dev_alloc(&m.w1x3, x3.size() * 2);
        if (e == hipSuccess) e = hipMemcpy(m.w1x3, x3.data(), x3.size() * 2, hipMemcpyHostToDevice);
        if (e != hipSuccess) { model_free(m); return hip_fail(e, "model upload"); }
        m.bytes += x3.size() * 2;
    }
    // FP8 hidden biases are stored in accumulator units, b / (s_a s_w)
    std::vector<float> bias(2 * H + CP, 0.0f);
    for (int k = 0; k < H; ++k) {
        bias[k] = p == TANG_FP8 ? (float)((double)b[0][k] / (double)m.deq[0]) : b[0][k];
        bias[H + k] = p == TANG_FP8 ? (float)((double)b[1][k] / (double)m.deq[1]) : b[1][k];
    }
    for (int k = 0; k < C; ++k) bias[2 * H + k] = b[2][k];
    hipError_t e = dev_alloc(&m.bias, bias.size() * 4);
    if (e == hipSuccess) e = hipMemcpy(m.bias, bias.data(), bias.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) { model_free(m); return hip_fail(e, "bias upload"); }
    m.bytes += bias.size() * 4;
    m.loaded = 1;
    model_free(rs->model);
    rs->model = m;
    rs->version++;
    return TANG_OK;
}

namespace {

template <int PREC, int H, int NT, int LDSM, int WAVES = 8, int OUTB = 1>
hipError_t launch_t(const ModelDev& m, const tang_header_t* d_hdr, uint32_t n, uint32_t* cand,
                    float* logits, uint16_t* cand16, hipStream_t s, const uint32_t* live) {
    using F = typename FragT<PREC>::T;
    constexpr int KB = FragT<PREC>::KB;
    constexpr size_t n1 = (H / 16) * (kInPad / KB) * 64, n2 = (H / 16) * (H / KB) * 64,
                     n3 = 2 * (H / KB) * 64;
    const size_t lds = ((LDSM & 1) ? n1 : 0) * sizeof(F) + ((LDSM & 2) ? n2 : 0) * sizeof(F) +
                       ((LDSM & 4) ? n3 : 0) * sizeof(F) + (2 * H + kOutPad * OUTB) * sizeof(float) +
                       (PREC == TANG_FP8 ? 256 * 8 : 256 * 16);  // bit table (BF16's for FP32)
    auto kern = k_mlp<PREC, H, NT, LDSM, WAVES, OUTB>;
    static int attr_done = 0;  // per instantiation
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)lds);
        if (e != hipSuccess) return e;
        attr_done = 1;
    }
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern, 64 * WAVES, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const uint32_t tiles = (n + 16 * NT - 1) / (16 * NT);
    const uint32_t want = (tiles + WAVES - 1) / WAVES;
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(want, (uint32_t)(cus * per_cu)));
    MlpArgs a;
    a.n_out = m.n_out;
    a.topk = m.topk;
    a.n3 = m.w3frags;
    a.nbias = 2 * H + kOutPad * ((m.n_out + kOutPad - 1) / kOutPad);
    for (int l = 0; l < 3; ++l) { a.deq[l] = m.deq[l]; a.inv_a[l] = m.inv_a[l]; }
    for (int l = 0; l < 2; ++l) { a.rq[l] = m.rq[l]; a.rb[l] = 448.0f * m.rq[l]; }
    hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * WAVES), lds, s,
                       reinterpret_cast<const uint4*>(d_hdr), n, (const F*)m.w[0], (const F*)m.w[1],
                       (const F*)m.w[2], (const u32x4*)m.w1x3, m.bias, a, cand, logits, cand16, live);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_mlp(const tang_ruleset_t* rs, const tang_header_t* d_hdr, size_t n,
                      uint32_t* d_cand_packed, float* d_logits, uint16_t* d_cand16, hipStream_t s, bool beside_search,
                      const uint32_t* d_live) {
    const ModelDev& m = rs->model;
    if (m.kind == 1) {
        if (d_live) return hipErrorInvalidValue;
        return launch_resnet(rs, d_hdr, n, d_cand_packed, d_logits, d_cand16, s);
    }
    const size_t chunk = (size_t)1 << 30;
    if (d_live && n > chunk) return hipErrorInvalidValue;
    for (size_t base = 0; base < n; base += chunk) {
        const uint32_t k = (uint32_t)std::min(chunk, n - base);
        const tang_header_t* h = d_hdr + base;
        uint32_t* c = d_cand_packed ? d_cand_packed + base : nullptr;
        float* lg = d_logits ? d_logits + base * (size_t)m.n_out : nullptr;
        uint16_t* c8 = d_cand16 ? d_cand16 + base * (size_t)m.topk : nullptr;
        hipError_t e;
        // LDSM: which layers' fragments sit in LDS (bit l = layer l) -- 160 KB per CU.
        // FP32 reads its input layer's BF16 planes from L2 (bit 0 unused).
        // At H = 256 the predictor alone runs BF16 as 8 waves of 64 headers (NT = 4: each
        // weight fragment read from LDS serves four header tiles; 254 VGPRs) and FP8 as 16
        // waves of 32 (its 126 VGPRs allow four per SIMD: 1.81 -> 1.71 ms against 12
        // waves); beside a chunked classify's search both run 8 waves of 32 headers,
        // so that search waves fit on every SIMD next to them (measured per 16M headers:
        // BF16 alone 2.56 ms with 12 waves of 32, 2.44 ms with 8 of 64; chunked classify
        // unchanged by the alone variant). Below 2^20 headers (serving batches) BF16 keeps
        // 12 waves of 32: a workgroup of 512 headers would leave half of the CUs idle on a
        // 65,536-header batch.
        // More than 32 tuples: up to 16 blocks of 32 classes, W3 read from L2.
        const bool wide = m.n_out > kOutPad;
        if (wide) {
            if (m.prec == TANG_FP32 && m.hidden == 128) e = launch_t<TANG_FP32, 128, 2, 2, 8,16>(m, h, k, c, lg, c8, s, d_live);
            else if (m.prec == TANG_FP32) e = launch_t<TANG_FP32, 256, 1, 0, 8,16>(m, h, k, c, lg, c8, s, d_live);
            else if (m.prec == TANG_BF16 && m.hidden == 128) e = launch_t<TANG_BF16, 128, 2, 3, 8,16>(m, h, k, c, lg, c8, s, d_live);
            else if (m.prec == TANG_BF16) e = launch_t<TANG_BF16, 256, 2, 2, 8,16>(m, h, k, c, lg, c8, s, d_live);
            else if (m.hidden == 128) e = launch_t<TANG_FP8, 128, 2, 3, 8,16>(m, h, k, c, lg, c8, s, d_live);
            else e = launch_t<TANG_FP8, 256, 2, 3, 8,16>(m, h, k, c, lg, c8, s, d_live);
        }
        else if (m.prec == TANG_FP32 && m.hidden == 128) e = launch_t<TANG_FP32, 128, 2, 6>(m, h, k, c, lg, c8, s, d_live);
        else if (m.prec == TANG_FP32) e = launch_t<TANG_FP32, 256, 1, 0>(m, h, k, c, lg, c8, s, d_live);
        else if (m.prec == TANG_BF16 && m.hidden == 128) e = launch_t<TANG_BF16, 128, 2, 7>(m, h, k, c, lg, c8, s, d_live);
        else if (m.prec == TANG_BF16 && beside_search) e = launch_t<TANG_BF16, 256, 2, 6, 8>(m, h, k, c, lg, c8, s, d_live);
        else if (m.prec == TANG_BF16 && k < (1u << 20)) e = launch_t<TANG_BF16, 256, 2, 6, 12>(m, h, k, c, lg, c8, s, d_live);
        else if (m.prec == TANG_BF16) e = launch_t<TANG_BF16, 256, 4, 6, 8>(m, h, k, c, lg, c8, s, d_live);
        else if (m.hidden == 128) e = launch_t<TANG_FP8, 128, 2, 7>(m, h, k, c, lg, c8, s, d_live);
        else if (beside_search) e = launch_t<TANG_FP8, 256, 2, 7, 8>(m, h, k, c, lg, c8, s, d_live);
        else e = launch_t<TANG_FP8, 256, 2, 7, 16>(m, h, k, c, lg, c8, s, d_live);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tang
