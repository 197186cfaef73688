// Internal declarations of the gfx950 packet classifier: device data layout, the slot
// hash, the ruleset object and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/tang.h"

namespace tang {

// ---------------------------------------------------------------------------------------
// Device layout.
//
// Slot (16 B): one bucket of the global open-addressing table. The key is the full
// (tuple, SIP & mask_t, DIP & mask_t), so an answer never depends on the hash function.
//   tl = tuple << 20 | bucket length; kEmptyTL marks a never-used slot.
//   off = first record of the bucket in the record array.
struct alignas(16) Slot {
    uint32_t ms, md, tl, off;
};
constexpr uint32_t kEmptyTL = 0xFFFFFFFFu;
constexpr uint32_t kTlShift = 20;
constexpr uint32_t kMaxBucketLen = (1u << kTlShift) - 1u;

// Long buckets are split. A bucket that would hold more than kSplitAt rules keeps its
// slot only as a marker (len 0, off = kSplit | bucket index); its rules move to four
// sub-lists stored in the same table under keys (tuple | kind << 8, bucket index, value):
//   kSubDp    rules with an exact DP, value = that DP
//   kSubSp    rules with an exact SP (DP not exact), value = that SP
//   kSubProto rules with an exact protocol and no exact port, value = the protocol
//   kSubRest  every other rule, value 0
// A header reads the four lists its own DP, SP and protocol select; each list is in
// (priority, id) order, so the first match of each is its best and the minimum of the
// four is the bucket's best. Rules that cannot match the header are never scanned.
constexpr uint32_t kSplit = 0x80000000u;
constexpr uint32_t kSplitAt = 16;
enum : uint32_t { kSubDp = 1, kSubSp = 2, kSubProto = 3, kSubRest = 4 };
constexpr uint32_t kKindShift = 9;   // tuples < 512; tuple | kind << 9 fits the slot's 12 bits

// Conflict masks: one word per rule (in the record) for rulesets of at most 32 tuples;
// wider ones keep a side array indexed like the records, kMaskWords words per rule for
// at most 256 tuples and kMaxWords for more (up to TANG_MAX_TUPLES).
constexpr int kMaskWords = 8;
constexpr int kMaxWords = TANG_MAX_TUPLES / 32;
// Mask words for a tuple count, and the tuple limit of a mask width.
inline uint32_t words_for(size_t tuples) {
    return tuples <= 32 ? 1u : tuples <= 32u * kMaskWords ? (uint32_t)kMaskWords : (uint32_t)kMaxWords;
}
inline size_t tuple_limit(uint32_t nw) { return 32u * (size_t)nw; }
// Candidate tuples in the predictor's output word: one byte each up to 256 tuples (at
// most 4 candidates), 16 bits each above (at most 2).
__host__ __device__ inline uint32_t cand_bits(int n_tuples) { return n_tuples > 256 ? 16u : 8u; }
inline int max_topk(int n_tuples) {
    const int k = n_tuples > 256 ? 2 : TANG_MAX_TOPK;
    return k < n_tuples ? k : n_tuples;
}

// Rec (32 B): one rule as the bucket scan reads it, hot half first. The scan reads the
// first 16 bytes of each record (one load): ports, priority and the protocol/length
// word decide a match for a rule held by its own tuple. The second half is read only
// for a match (its id and conflict mask), a priority tie (the id breaks it), or a rule
// held by a coarser tuple than its own signature (its prefixes must be checked).
//   sp, dp   : lo | hi << 16 (inclusive)
//   prio     : priority; (prio, id) is the key, kDead in both marks a vacated record
//   meta     : proto (bits 0-7) | exact-proto (8) | prefix check (9) | sip_len (10-15)
//              | dip_len (16-21) | tuple (22-31)
//   sip, dip : prefix values, bits beyond the length zeroed
//   id       : rule id
//   cmask    : conflict tuples of a ruleset of at most 32 tuples (wider ones: side
//              array) -- tuples that hold a higher-priority rule whose box meets this
//              rule's box (a superset after deletes)
struct alignas(16) Rec {
    uint32_t sp, dp, prio, meta, sip, dip, id, cmask;
};
constexpr uint32_t kDead = 0xFFFFFFFFu;

__host__ __device__ inline uint32_t meta_pack(uint32_t sl, uint32_t dl, uint32_t proto,
                                              uint32_t exact, uint32_t tuple, uint32_t check) {
    return proto | (exact << 8) | (check << 9) | (sl << 10) | (dl << 16) | (tuple << 22);
}
__host__ __device__ inline uint32_t meta_proto(uint32_t m) { return m & 255u; }
__host__ __device__ inline uint32_t meta_exact(uint32_t m) { return (m >> 8) & 1u; }
__host__ __device__ inline uint32_t meta_check(uint32_t m) { return (m >> 9) & 1u; }
__host__ __device__ inline uint32_t meta_sl(uint32_t m) { return (m >> 10) & 63u; }
__host__ __device__ inline uint32_t meta_dl(uint32_t m) { return (m >> 16) & 63u; }
__host__ __device__ inline uint32_t meta_tuple(uint32_t m) { return m >> 22; }

// Prefix mask of length l (0..32): the top l bits; l = 0 gives 0 (no shift by 32).
__host__ __device__ inline uint32_t pmask(uint32_t l) {
    return l == 0 ? 0u : (0xFFFFFFFFu << (32u - l));
}

// Per-tuple data: masks and the smallest (priority, id) key of any rule ever placed in
// the tuple (a lower bound after deletes, used to stop searching tuples early).
struct TupleDev {
    uint32_t smask, dmask, best_prio, best_id;
};
// Filter groups: the tuples whose longer prefix is the SIP (sip_len >= dip_len) share a
// group per SIP length, the others a group per DIP length; tuple (0, 0), whose only
// possible key always has a bucket, has none. At most 64 groups (32 lengths per field).
constexpr int kMaxGroups = 64;
constexpr uint32_t kNoGroup = 0xFFu;
struct TupleTable {
    TupleDev t[TANG_MAX_TUPLES];
    uint16_t order[TANG_MAX_TUPLES]; // tuple indices by ascending best key
    uint32_t rank_prio[TANG_MAX_TUPLES], rank_id[TANG_MAX_TUPLES];  // best keys in that order
    // prefix[k]: the k tuples of lowest best key, as mask words
    uint32_t prefix[TANG_MAX_TUPLES + 1][kMaxWords];
    uint32_t n;                       // number of tuples
    uint32_t all_mask[kMaxWords];     // bits of all tuples
    uint32_t slot_mask;               // slots - 1
    uint32_t filter_mask;             // filter blocks - 1
    uint32_t nw;                      // mask words of this ruleset (1, kMaskWords or kMaxWords)
    uint8_t gid[TANG_MAX_TUPLES];     // filter group of each tuple (kNoGroup: none)
    uint32_t ngroups;
    uint32_t gkey[kMaxGroups];        // side (bit 6: 1 = DIP) | prefix length (bits 0-5)
    uint32_t gmask[kMaxGroups][kMaxWords];  // tuples of each group
    uint32_t nogroup[kMaxWords];      // tuples without a group (always pass)
};

// Key hash: two chained MurmurHash3 32-bit finalisers (fmix32, Appleby, public domain),
// first over the masked SIP salted by the tuple index, then over that result xor the
// masked DIP. Each stage is a bijection, so structured keys (prefixes whose only varying
// bits are the top byte) do not collapse. The low half of the result picks the slot.
// The bucket filter uses its own cheaper hashes (filter_block / filter_bits below).
__host__ __device__ inline uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}
__host__ __device__ inline uint64_t key_hash(uint32_t t, uint32_t ms, uint32_t md) {
    const uint32_t h = fmix32(fmix32(ms + (t + 1u) * 0x9E3779B9u) ^ md);
    uint32_t f = (h ^ (h >> 15)) * 0x2C1B3C6Du;
    f ^= f >> 12;
    return ((uint64_t)f << 32) | h;
}
__host__ __device__ inline uint32_t slot_of(uint64_t h) { return (uint32_t)h; }
// Bucket filter, blocked by prefix group. A main bucket (t, ms, md) of a tuple with
// lengths (ls, ld) belongs to the tuple's filter group: the SIP group of length ls when
// ls >= ld, else the DIP group of length ld. The group value v (ms or md) picks one
// 64-bit block, filter_block(gkey, v); the other masked field o (md or ms) and the tuple
// pick two bits in it, filter_bits(t, o) (a blocked Bloom filter with two probes: with
// about two buckets per block a tuple passes by chance 0.3% of the time instead of 3% --
// it matters when a packet tests a hundred tuples). A header then reads one block per
// group for all the tuples of that group (at most 5 blocks for the 25 tuples of five
// lengths per field), where a bit per tuple took one load each. A clear bit means no
// bucket; a set pair may be a collision, which only costs a slot walk. Placement never
// affects answers.
__host__ __device__ inline uint32_t filter_block(uint32_t gkey, uint32_t v) {
    uint32_t x = v ^ ((gkey + 1u) * 0x9E3779B9u);
    x *= 0x85EBCA6Bu;
    x ^= x >> 15;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return x;
}
// The two bit positions (0..63) in bits 0-5 and 8-13.
__host__ __device__ inline uint32_t filter_bits(uint32_t t, uint32_t o) {
    const uint32_t h = (o ^ ((t + 1u) * 0x7FEB352Du)) * 0x846CA68Bu;
    return (h >> 26) | (((h >> 18) & 63u) << 8);
}
__host__ __device__ inline uint32_t group_key_of(uint32_t ls, uint32_t ld) {
    return ls >= ld ? ls : (64u | ld);
}

// Device-side counters for tang_stats_t (kStatCopies copies, summed on the host).
struct StatsDev {
    unsigned long long packets, probes, slots, records, top1, fallbacks, nomatch, filters, steps,
        rounds;
};
constexpr int kStatCopies = 64;

// Rule box used by the conflict-mask kernels (key order), 32 B.
struct alignas(16) BoxDev {
    uint32_t slo, shi, dlo, dhi, sp, dp, pt, pos;  // pt = proto | exact << 8 | tuple << 16
};

// ---------------------------------------------------------------------------------------
// Model on the device.

constexpr int kMaxHidden = 256;
constexpr int kOutPad = 32;   // output classes padded to 2 MFMA tiles
constexpr int kInPad = 128;   // 104 input bits padded to 128

struct ModelDev {
    int loaded = 0;
    int kind = 0;     // 0: the plain 104 -> H -> H -> C network; 1: the residual network
    tang_precision_t prec = TANG_FP32;
    int hidden = 0;
    int n_out = 0;    // C
    uint32_t w3frags = 0;  // output-layer weight fragments (classes padded to 32-blocks)
    int topk = 1;
    // Weight fragments for the three layers in MFMA A-operand order, and biases.
    void* w[3] = {nullptr, nullptr, nullptr};
    size_t wbytes[3] = {0, 0, 0};
    // FP32 models: W1 as three BF16 planes (hi + mid + lo = W1 exactly) in BF16 fragment
    // order, for the input layer on BF16 MFMAs (its inputs are bits, so products are exact)
    void* w1x3 = nullptr;
    float* bias = nullptr;   // [hidden | hidden | 32] floats
    float deq[3] = {1, 1, 1};     // FP8: s_a * s_w per layer
    float inv_a[3] = {1, 1, 1};   // FP8: 1 / s_a per layer (layer 0 unused)
    float rq[2] = {1, 1};         // FP8 hidden layers: 2^-e, e the requantisation exponent
    // Residual network: input layer FP32 [512][8], BF16 layer weights, BF16 activation
    // workspace (three chunk buffers) and the event that orders calls sharing it.
    int n_blocks = 0;
    float* rin = nullptr;
    void* rw = nullptr;
    uint16_t* ws = nullptr;
    hipEvent_t ws_done = nullptr;
    mutable bool ws_used = false;
    size_t bytes = 0;
};

}  // namespace tang

// ---------------------------------------------------------------------------------------
// The ruleset object behind tang_ruleset_t.

struct tang_ruleset_s {
    struct HRule {
        tang_rule_t r;      // normalised
        uint32_t tuple;
        uint32_t bucket;
        uint32_t pos;       // record index on the device
        bool live;
    };
    struct Bucket {
        uint32_t t, ms, md;             // t | kind << kKindShift (kind 0: main bucket)
        uint32_t slot;
        uint32_t off, cap;
        std::vector<uint32_t> members;  // rule handles in (priority, id) order
        bool split = false;             // main bucket whose rules live in sub-lists
    };
    struct BKey {
        uint32_t t, ms, md;
        bool operator==(const BKey& o) const { return t == o.t && ms == o.ms && md == o.md; }
    };
    struct BKeyHash {
        size_t operator()(const BKey& k) const {
            return (size_t)tang::key_hash(k.t, k.ms, k.md);
        }
    };

    int device = TANG_HOST_ONLY;
    std::vector<HRule> rules;                      // handle-indexed, never shrinks
    std::unordered_map<uint32_t, uint32_t> id2h;   // live id -> handle
    size_t n_live = 0;
    size_t n_coarse = 0;   // live rules held by a tuple coarser than their own signature
    std::vector<std::pair<uint8_t, uint8_t>> sigs; // tuple signatures
    std::vector<uint64_t> tuple_best;              // lower bound on keys per tuple
    std::vector<Bucket> buckets;
    std::unordered_map<BKey, uint32_t, BKeyHash> bucket_of;
    std::vector<tang::Slot> slots;                 // host mirror of the slot table
    std::vector<uint32_t> filter;                  // host mirror of the bucket filter (2 words per block)
    uint32_t rec_used = 0, rec_cap = 0;
    uint32_t nw = 1;   // conflict-mask words per rule (fixed at build: words_for(tuples))

    // device state
    tang::Slot* d_slots = nullptr;
    uint32_t* d_filter = nullptr;
    tang::Rec* d_recs = nullptr;
    uint32_t* d_cmask = nullptr;   // nw > 1: nw words per record position
    tang::TupleTable* d_tt = nullptr;
    tang::StatsDev* d_stats = nullptr;
    hipStream_t upd_stream = nullptr;
    tang::ModelDev model;
    std::mutex stats_mu;
    mutable std::mutex ws_mu;  // enqueueing of residual-model launches (shared workspace)
    // Chunked classify: the searches of a large batch run on this stream (created on first
    // use, default priority), each after its chunk's model on the caller's stream.
    std::mutex pipe_mu;
    hipStream_t pipe_stream = nullptr;
    std::vector<hipEvent_t> pipe_events;
    uint64_t version = 0;   // bumped by every change that captured launches depend on
    bool failed = false;    // an update's device flush failed: host and device disagree

    size_t device_bytes() const;
};

namespace tang {

// Error reporting (thread-local message + code).
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
#define TANG_HIP(call)                                         \
    do {                                                       \
        hipError_t _e = (call);                                \
        if (_e != hipSuccess) return ::tang::hip_fail(_e, #call); \
    } while (0)

// Host tuple space (tss.cpp).
int validate_rule(const tang_rule_t& r);
tang_rule_t normalise(const tang_rule_t& r);
inline uint64_t key_of(const tang_rule_t& r) { return ((uint64_t)r.priority << 32) | r.id; }
int build_host(tang_ruleset_t* rs, const tang_rule_t* rules, size_t n);
int upload_all(tang_ruleset_t* rs);
TupleTable make_tuple_table(const tang_ruleset_t* rs);
Rec make_rec(const tang_ruleset_t* rs, uint32_t h);
int apply_insert(tang_ruleset_t* rs, const tang_rule_t* rules, size_t n);
int apply_delete(tang_ruleset_t* rs, const uint32_t* ids, size_t n);

// Internal device memory: through the caller's allocator when one is set
// (tang_set_allocator), else hipMalloc / hipFree; a block is released through the
// allocator that provided it.
hipError_t dev_alloc(void** p, size_t bytes);
hipError_t dev_release(void* p);
template <class T>
inline hipError_t dev_alloc(T** p, size_t bytes) {
    return dev_alloc(reinterpret_cast<void**>(p), bytes);
}

// Kernel launchers (k_classify.hip, k_build.hip, k_mlp.hip).
// d_live (optional): a device word holding the live header count, read by the kernels at
// their start; lanes and workgroups past min(n, *d_live) do nothing. A launch recorded
// once into a graph for n headers then serves any smaller batch without padding.
hipError_t launch_classify(const tang_ruleset_t* rs, const tang_header_t* d_hdr,
                           uint32_t* d_out, size_t n, int kcand, hipStream_t s, bool stats,
                           const uint32_t* d_live = nullptr);
hipError_t launch_conflict_build(const BoxDev* d_boxes, size_t n, Rec* d_recs, uint32_t* d_cmask,
                                 uint32_t nw, const uint32_t* all_mask,
                                 hipStream_t s);
hipError_t launch_conflict_update(Rec* d_recs, uint32_t* d_cmask, uint32_t nw, uint32_t rec_used,
                                  const uint32_t* d_new_pos, uint32_t n_new, hipStream_t s);
hipError_t launch_move_records(Rec* d_recs, const Rec* d_src_recs, const uint32_t* d_src,
                               const uint32_t* d_dst, uint32_t n, Rec* d_stage, hipStream_t s);
// nw > 1: the mask rows move with their records (the same src / dst lists; new sources
// get zero rows), through a stage of n rows.
hipError_t launch_move_masks(uint32_t* d_cmask, uint32_t nw, const uint32_t* d_src,
                             const uint32_t* d_dst, uint32_t n, uint32_t* d_stage, hipStream_t s);
hipError_t launch_scatter_slots(Slot* d_slots, const uint32_t* d_idx, const Slot* d_val,
                                uint32_t n, hipStream_t s);
// Batches of at least two chunks of this many headers, with a BF16 or FP8 model and no
// stats, are classified chunk by chunk with the model and the search on two streams.
constexpr size_t kPipeChunk = (size_t)1 << 21;
// Largest batch of tang_classify_host_noalloc (its static staging: 5 MiB per GPU).
constexpr size_t kNoAllocMaxHeaders = (size_t)1 << 18;
// tang_classify's body; allow_chunks = false keeps every launch on stream s (for callers
// that capture the launches into a graph).
// d_live: as for launch_classify (with a plain MLP or no model; not with stats).
int classify_async(tang_ruleset_t* rs, const tang_header_t* d_hdr, uint32_t* d_rule_id, size_t n,
                   hipStream_t s, tang_stats_t* stats, bool allow_chunks,
                   const uint32_t* d_live = nullptr);
// beside_search: the launch overlaps a search on another stream (the chunked classify),
// so the predictor leaves room on every SIMD for search waves.
hipError_t launch_mlp(const tang_ruleset_t* rs, const tang_header_t* d_hdr, size_t n,
                      uint32_t* d_cand_packed, float* d_logits, uint16_t* d_cand16,
                      hipStream_t s, bool beside_search = false, const uint32_t* d_live = nullptr);
int search_host(const tang_ruleset_t* rs, const tang_header_t* hdr, const uint32_t* cand,
                uint32_t* out, size_t n, uint32_t kcand, uint32_t threads, bool exact,
                tang_stats_t* stats);
int resnet_prepare(tang_ruleset_t* rs, const tang_resnet_desc_t* d, const float* const* W,
                   const float* const* b, tang_precision_t p);
hipError_t launch_resnet(const tang_ruleset_t* rs, const tang_header_t* d_hdr, size_t n,
                         uint32_t* cand, float* logits, uint16_t* cand16, hipStream_t s);
int model_prepare(tang_ruleset_t* rs, const tang_mlp_desc_t* d, const float* const* W,
                  const float* const* b, tang_precision_t p, const float* act_scales);
void model_free(ModelDev& m);

}  // namespace tang
