/*
 * tang.h -- C ABI of an MI355X (gfx950) batched 5-field packet classifier.
 *
 * The method is TaNG's two-stage classification (Sec. 5.1.1): a small MLP reads each
 * packet header and predicts which tuple of a tuple space (Sec. 4.3) holds the answer;
 * the packet's SIP/DIP are truncated to that tuple's prefix lengths, hashed, and the
 * hashed bucket's rules are checked in (priority, id) order. Unlike the paper, which accepts a
 * rare lower-priority answer (Sec. 5.1.1, Sec. 8), this library certifies every
 * answer: after the predicted tuples it probes each tuple that holds a higher-priority
 * rule overlapping the match found (a per-rule "conflict mask"), or every remaining
 * tuple when nothing matched. The returned id is therefore always the exact
 * highest-priority match, whatever the model predicts.
 *
 * Conventions shared by every call:
 *   - Every function returns int: 0 on success or a negative TANG_E* code. No C++
 *     exception crosses this boundary. tang_last_error() returns a message for the
 *     last failure on the calling thread.
 *   - "device pointer" means memory the caller allocated on the ruleset's GPU (for
 *     example a torch tensor's data_ptr); "host pointer" means ordinary CPU memory.
 *   - A stream argument is a hipStream_t passed as void* (NULL = the null stream).
 *   - Input arrays are deep-copied; the caller keeps ownership of everything it passes.
 *   - The library owns only its internal device memory (hipMalloc'd on the ruleset's
 *     device, or taken from the caller's allocator, see tang_set_allocator; freed by
 *     tang_ruleset_destroy, model reloads and server destruction).
 */
#ifndef TANG_H
#define TANG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TANG_NO_MATCH 0xFFFFFFFFu /* rule_id when no rule matches (no default rule) */
#define TANG_HOST_ONLY (-1)       /* device argument: build host structures only */
#define TANG_MAX_TUPLES 512       /* conflict masks up to 16 words */
#define TANG_MAX_TOPK 4           /* 2 for rulesets of more than 256 tuples */
#define TANG_MAX_LAYERS 8

enum {
    TANG_OK = 0,
    TANG_EINVAL = -1,    /* bad argument or rule field */
    TANG_ENOMEM = -2,    /* host or device allocation failed, or a capacity is exceeded */
    TANG_ENOTFOUND = -3, /* delete of an id that is not live */
    TANG_EEXIST = -4,    /* insert of an id that is already live (or repeated in a batch) */
    TANG_EDEVICE = -5,   /* a HIP call failed */
    TANG_EBUSY = -6,     /* server: request refused or still running */
    TANG_ETIMEOUT = -7   /* server: wait timed out */
};

/*
 * A rule (Sec. 2.1): SIP and DIP prefixes (value + length 0..32; bits beyond the
 * length are ignored and normalised to zero), inclusive port ranges lo <= hi, and a
 * protocol that is exact (proto_mask = 0xFF) or wildcard (proto_mask = 0). Priorities
 * follow Table 1: a lower number is a higher priority. Equal priorities are ordered by
 * the lower id. id must be unique among live rules and != TANG_NO_MATCH. 28 bytes.
 */
typedef struct tang_rule_s {
    uint32_t sip, dip;
    uint32_t priority;
    uint32_t id;
    uint16_t sp_lo, sp_hi, dp_lo, dp_hi;
    uint8_t sip_len, dip_len;
    uint8_t proto, proto_mask;
} tang_rule_t;

/* A packet header, 16 bytes (13 used): SIP, DIP, SP, DP, protocol, 3 pad bytes. */
typedef struct tang_header_s {
    uint32_t sip, dip;
    uint16_t sp, dp;
    uint8_t proto;
    uint8_t pad[3];
} tang_header_t;

typedef enum { TANG_FP32 = 0, TANG_BF16 = 1, TANG_FP8 = 2 } tang_precision_t;

/*
 * The predictor (Sec. 6.1, plain form without residual blocks): n_layers Linear
 * layers, dims[0] -> dims[1] -> ... -> dims[n_layers], ReLU after every layer but the
 * last. dims[0] must be 104: the header's bits, most significant first, over SIP(32)
 * DIP(32) SP(16) DP(16) PROTO(8), each as 0.0 or 1.0. dims[n_layers] must equal
 * tang_ruleset_num_tuples() (1..TANG_MAX_TUPLES). Supported now: n_layers = 3 with equal hidden widths
 * 128 or 256. topk (1..4; 1..2 above 256 tuples) is how many top-scoring tuples are
 * probed before certification; equal scores go to the lower tuple index (argmax of
 * Sec. 6.1 for 1).
 */
typedef struct tang_mlp_desc_s {
    uint32_t n_layers;
    uint32_t dims[TANG_MAX_LAYERS + 1];
    uint32_t topk;
} tang_mlp_desc_t;

/* Optional per-call counters (tang_classify with a non-NULL stats; synchronises). */
typedef struct tang_stats_s {
    uint64_t packets;     /* packets classified */
    uint64_t probes;      /* hash-table probes (one per tuple searched) */
    uint64_t slots;       /* hash slots read */
    uint64_t records;     /* rule records compared */
    uint64_t top1_hits;   /* answer lies in the first predicted tuple */
    uint64_t fallbacks;   /* nothing matched in the predicted tuples */
    uint64_t no_match;    /* packets with no matching rule at all */
    uint64_t filter_checks;  /* bucket-filter bits read (one per tuple reached) */
    uint64_t wave_steps;     /* per packet: most filter-passing tuples of a packet in its wave */
    uint64_t wave_rounds;    /* per packet: filter-sweep batches (8 tuples) of its wave */
} tang_stats_t;

typedef struct tang_ruleset_s tang_ruleset_t;

/*
 * Build a ruleset: tuple space with tuples numbered by first appearance over rules in
 * ascending (priority, id) order (Table 1), one open-addressing hash table of buckets
 * keyed by (tuple, SIP & mask, DIP & mask), each bucket's rules sorted by (priority,
 * id) (Sec. 4.3, 5.1.1), and per-rule conflict masks computed on the GPU.
 * device: GPU ordinal, or TANG_HOST_ONLY to build only the host tuple space (for
 * inspection; such a ruleset cannot classify or load a model).
 * rules: host pointer to n rules (n may be 0). *out receives the handle.
 * Errors: EINVAL (a length > 32, lo > hi, proto_mask not 0/0xFF, id = TANG_NO_MATCH,
 * more than TANG_MAX_TUPLES signatures), EEXIST (repeated id), ENOMEM, EDEVICE.
 */
int tang_ruleset_create(int device, const tang_rule_t* rules, size_t n, tang_ruleset_t** out);
void tang_ruleset_destroy(tang_ruleset_t* rs);

/*
 * Number of tuples C (the model's output width, Sec. 6.1) and the signature of tuple t:
 * its (SIP length, DIP length), tuples numbered by first appearance over the rules in
 * ascending (priority, id) order as in Table 1 (Sec. 4.3). EINVAL for t >= C.
 */
uint32_t tang_ruleset_num_tuples(const tang_ruleset_t* rs);
int tang_ruleset_tuple(const tang_ruleset_t* rs, uint32_t t, uint8_t* sip_len, uint8_t* dip_len);
/* Number of live rules. */
size_t tang_ruleset_num_rules(const tang_ruleset_t* rs);
/* Tuple that holds live rule `id` (ENOTFOUND if none). */
int tang_ruleset_rule_tuple(const tang_ruleset_t* rs, uint32_t id, uint32_t* tuple);
/*
 * Conflict mask of live rule `id` (bit t = tuple t), read back from the device
 * (synchronises): tang_ruleset_conflict_mask gives tuples 0..31; _words gives n_words
 * words (word w = tuples 32w..32w+31), zero past the ruleset's mask width. The mask width
 * is fixed when the ruleset is built: one word per rule for at most 32 tuples, 8 words
 * for at most 256, 16 words above (up to TANG_MAX_TUPLES). An insertion that would
 * append a tuple past the width's limit (the 33rd, 257th or 513th) fails with EINVAL;
 * rebuilding the ruleset from tang_ruleset_export lifts it.
 */
int tang_ruleset_conflict_mask(tang_ruleset_t* rs, uint32_t id, uint32_t* mask);
int tang_ruleset_conflict_mask_words(tang_ruleset_t* rs, uint32_t id, uint32_t* words,
                                     uint32_t n_words);
/* Device bytes held by the ruleset (tables, records, model). */
int tang_ruleset_device_bytes(const tang_ruleset_t* rs, size_t* bytes);
/* Stream on which updates are applied (default: the null stream). */
int tang_ruleset_set_stream(tang_ruleset_t* rs, void* stream);

/*
 * Drift of the tuple space under updates (Sec. 5.2.2): the number of live rules that an
 * insert placed in a tuple coarser than their own (SIP, DIP) length signature (restricted
 * insertion, Sec. 5.2.1), counted since the ruleset was built; a delete of such a rule
 * lowers it. The deferred-update policy compares it with its threshold theta.
 */
int tang_ruleset_coarse_rules(const tang_ruleset_t* rs, size_t* count);
/*
 * The live rules, normalised (host bits below each prefix cleared), in ascending
 * (priority, id) order: what a full rebuild of the tuple space starts from (Sec. 5.2.2).
 * out == NULL: only *n = number of live rules. Otherwise out (host) must hold cap >= *n
 * rules, else EINVAL.
 */
int tang_ruleset_export(const tang_ruleset_t* rs, tang_rule_t* out, size_t cap, size_t* n);

/*
 * Load the predictor of Sec. 6.1 (plain form), weights deep-copied. W[l] is a host
 * pointer to dims[l+1] x dims[l] floats, row-major [out][in] (PyTorch
 * nn.Linear.weight); b[l] to dims[l+1] floats.
 * precision: FP32 (weights as given), BF16 (weights and each layer's input rounded to
 * bfloat16, nearest-even), FP8 (OCP E4M3 with static per-layer activation scales
 * act_scales[l] for l >= 1, act_scales[0] ignored since the input bits are exact;
 * inputs saturate at +-448; the output layer's weight scale is amax|W|/448, a hidden
 * layer's that scale raised by a factor in [1, 2) until s_w * act_scales[l] /
 * act_scales[l + 1] is a power of two, 2^e, so the layer's output is requantised by an
 * exact scaling; EINVAL if |e| > 100). Accumulation is FP32 and biases stay FP32 in every
 * precision. act_scales must be NULL unless precision is FP8.
 * Replaces any previously loaded model. Without a model, classify probes all tuples.
 */
int tang_model_load(tang_ruleset_t* rs, const tang_mlp_desc_t* desc, const float* const* W,
                    const float* const* b, tang_precision_t precision, const float* act_scales);
/* Drop the loaded model (of either kind); classify then probes every tuple. */
int tang_model_unload(tang_ruleset_t* rs);

/*
 * The paper's own predictor (Sec. 6.1 with residual blocks, Eq. 1; sizes of Sec. 7.1) on
 * its model input (Sec. 6.2): the header cut into seven 16-bit chunks (SIP high, SIP low,
 * DIP high, DIP low, SP, DP, PROTO), each divided by 65535; FC(7 -> width) + ReLU; then
 * n_blocks blocks x <- relu(relu(x w1 + b1) w2 + b2 + x); then FC(width -> C); top-k.
 * W / b: 2 + 2 n_blocks host pointers in nn.Linear layout [out][in]: W[0] width x 7,
 * W[1 + 2k] and W[2 + 2k] (block k's two layers) width x width, W[last] C x width.
 * Precision: BF16 only (the input layer is computed in FP32; every later layer's weights
 * and inputs are rounded to bfloat16, nearest-even; FP32 accumulation and biases).
 * Deep copy; replaces any loaded model. The library also allocates a 192 MB activation
 * workspace (three buffers of 65,536 headers x 512 BF16); calls that use this model on
 * one ruleset are ordered on the device through an event, whatever their streams.
 * Errors: EINVAL (width != 512, n_blocks outside 1..16, n_out != C, topk outside
 * 1..min(4, C), precision not BF16, NULL pointers), ENOMEM, EDEVICE.
 */
typedef struct tang_resnet_desc_s {
    uint32_t width;     /* neurons per FC layer: 512 */
    uint32_t n_blocks;  /* residual blocks (the paper uses 6) */
    uint32_t n_out;     /* C: the number of tuples */
    uint32_t topk;      /* candidates per header, 1..min(4, C) */
} tang_resnet_desc_t;
int tang_model_load_resnet(tang_ruleset_t* rs, const tang_resnet_desc_t* desc,
                           const float* const* W, const float* const* b,
                           tang_precision_t precision);

/*
 * Classify n headers (Sec. 2.1 problem statement; the two stages of Sec. 5.1.1, with
 * every answer certified): d_rule_id[i] = id of the highest-priority live rule matching
 * d_hdr[i], or TANG_NO_MATCH. d_hdr, d_rule_id: device pointers on the ruleset's GPU,
 * caller-owned, valid until the stream has passed this work. Asynchronous on `stream`
 * unless stats != NULL (then the counters are copied back and the call synchronises).
 * n = 0 is a no-op. Concurrent classify calls on any streams are allowed while no
 * update is in flight; order updates before classify through the streams.
 * With a BF16 or FP8 model loaded, no stats and n >= 2^22, the batch is processed in
 * chunks of 2^21 headers: each chunk's model runs on `stream` and its search on a stream
 * the ruleset owns (created on first use), overlapping the next chunk's model; `stream`
 * then waits for the last search, so completion is still observed through `stream`.
 * Chunked calls on one ruleset share that stream, so their searches run one after another.
 */
int tang_classify(tang_ruleset_t* rs, const tang_header_t* d_hdr, uint32_t* d_rule_id,
                  size_t n, void* stream, tang_stats_t* stats);
/*
 * The paper's own split as a comparison mode (Sec. 5.1.2: the GPU predicts, the CPU
 * searches): the search stage on the host tuple space, `threads` host threads. hdr,
 * rule_id: host arrays of n; cand: host array of n candidate words as tang_predict
 * writes them (candidate k in byte k), kcand of them per word (0: no prediction, the
 * ordered search over all tuples). exact = 0: the paper's search -- the best match of
 * the predicted tuples if any, else the ordered search over the remaining tuples by best
 * key (Sec. 5.1.1), so a lower-priority rule can be returned; exact != 0: the ordered
 * search always runs after the candidates, and the answer equals tang_classify's. Works
 * on host-only rulesets; must not overlap an update of the ruleset. Synchronous.
 * stats (optional): packets, probes, records, top1_hits, fallbacks, no_match.
 */
int tang_search_host(const tang_ruleset_t* rs, const tang_header_t* hdr, const uint32_t* cand,
                     uint32_t* rule_id, size_t n, uint32_t kcand, uint32_t threads, int exact,
                     tang_stats_t* stats);
/* Same with host pointers; copies in and out and synchronises. For tests and tools. */
int tang_classify_host(tang_ruleset_t* rs, const tang_header_t* hdr, uint32_t* rule_id,
                       size_t n, tang_stats_t* stats);
/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): tang_classify_host with the same
 * arguments, results and statistics, except that the headers and rule ids are staged in
 * a static device array the library holds on each GPU it runs on (5 MiB, kept until the
 * process ends) instead of device blocks allocated per call, so the call allocates
 * nothing. n is at most TANG_NOALLOC_MAX_HEADERS, else EINVAL. The batch is never split
 * over two streams. Calls that overlap on one GPU (from several threads, on any
 * rulesets) share the staging array and race: the caller serialises them.
 */
#define TANG_NOALLOC_MAX_HEADERS 262144u
int tang_classify_host_noalloc(tang_ruleset_t* rs, const tang_header_t* hdr, uint32_t* rule_id,
                               size_t n, tang_stats_t* stats);
/*
 * The two stages of tang_classify, callable one by one (Sec. 5.1.1): tang_predict runs
 * the model and writes each header's candidate tuples into d_io[i] (one byte per
 * candidate for rulesets of up to 256 tuples, 16 bits per candidate above; the first
 * candidate in the low bits); tang_search then probes, verifies and
 * certifies, reading those candidates from d_io and overwriting them with the rule ids.
 * Without a model tang_predict is an error and tang_search probes every tuple. Same
 * buffers, stream and concurrency rules as tang_classify; tang_search's stats as there.
 */
int tang_predict(tang_ruleset_t* rs, const tang_header_t* d_hdr, uint32_t* d_io, size_t n,
                 void* stream);
int tang_search(tang_ruleset_t* rs, const tang_header_t* d_hdr, uint32_t* d_io, size_t n,
                void* stream, tang_stats_t* stats);
/*
 * Predictor only: d_logits (device, may be NULL) receives n x C FP32 scores and d_cand
 * (device, may be NULL) n x topk tuple indices, 16 bits each. Asynchronous on `stream`.
 * Needs a model.
 */
int tang_mlp_forward(tang_ruleset_t* rs, const tang_header_t* d_hdr, size_t n, float* d_logits,
                     uint16_t* d_cand, void* stream);

/*
 * Immediate updates (Sec. 5.2.1). The tuple set is kept: an inserted rule goes to the
 * tuple with its own signature, else to the first tuple with the largest length sum
 * among those whose lengths are all <= the rule's (its prefixes are then checked in
 * the bucket scan); only if no tuple qualifies is a new tuple appended (the model
 * never predicts it; certification and the fallback still search it; past the mask
 * width's tuple limit, see tang_ruleset_conflict_mask_words, the batch fails with EINVAL).
 * A batch is validated as a whole before anything changes (all-or-nothing): insert
 * fails with EEXIST on a live or repeated id and EINVAL on a bad field; delete fails
 * with ENOTFOUND on an id that is not live. The device changes are enqueued on the
 * ruleset's stream (tang_ruleset_set_stream); later classify calls on that stream see
 * them. rules/ids: host pointers. An insert batch that would make one bucket list longer
 * than 2^20 - 1 rules (what a hash slot can describe) fails with ENOMEM before any change.
 * If the device part of an update fails (EDEVICE, or ENOMEM from a device allocation),
 * the host side already holds the batch: the ruleset then refuses every later call that
 * touches its device state with EDEVICE, and tang_ruleset_export still returns the live
 * rules (this batch included) to rebuild from.
 */
int tang_insert(tang_ruleset_t* rs, const tang_rule_t* rules, size_t n);
int tang_delete(tang_ruleset_t* rs, const uint32_t* ids, size_t n);

/* Message for the calling thread's last error ("" if none). */
const char* tang_last_error(void);

/*
 * Optional allocator for the library's internal device memory (tables, records, conflict
 * masks, model weights and workspaces, staging buffers, server slots), so that a caller's
 * pool (for example torch's caching allocator) can own it. alloc(bytes, device, ctx)
 * returns memory on HIP device `device` (the current device at the call), aligned to at
 * least 256 bytes, or NULL (the library then fails with TANG_ENOMEM); free(ptr, device,
 * ctx) returns it. Process-wide; alloc == NULL restores hipMalloc / hipFree. Each block
 * is returned through the allocator that provided it, even after a change, and only
 * after the device has finished its queued work (as hipFree would). The
 * callbacks may be called from any thread that calls into the library (and from the
 * serving loop's threads); they must not call back into it. Errors: EINVAL (exactly one
 * of alloc and free is NULL).
 */
typedef void* (*tang_alloc_fn)(size_t bytes, int device, void* ctx);
typedef void (*tang_free_fn)(void* ptr, int device, void* ctx);
int tang_set_allocator(tang_alloc_fn alloc, tang_free_fn free_fn, void* ctx);

/* ------------------------------------------------------------------------------------
 * Serving loop: continuous batching over several device-resident rulesets.
 * A persistent host thread admits submitted requests while in-flight packets and device
 * staging bytes stay within the configured limits, packs admitted requests of the same
 * ruleset into one batch, replays a captured HIP graph for that (ruleset, batch size
 * class), and completes each request with submit / admit / done timestamps.
 */
typedef struct tang_server_cfg_s {
    size_t mem_budget_bytes;        /* device staging bytes for in-flight batches */
    uint32_t max_inflight_packets;  /* admission limit on packets on the GPU */
    uint32_t n_streams;             /* concurrent batches (1..8) */
    uint32_t max_batch;             /* packets per launched batch (power of two) */
    uint32_t use_graphs;            /* 1: replay captured HIP graphs per size class */
} tang_server_cfg_t;

typedef struct tang_server_s tang_server_t;
typedef struct tang_req_s tang_req_t;

/*
 * Start a serving loop on HIP device `device` (one loop thread, three helper threads for
 * the host copies of large batches, n_streams stream slots with one issuing thread each
 * for the batches that move through the copy engines).
 * cfg may be NULL; zero fields take defaults: 4 streams, max_batch 65536, in-flight
 * packets n_streams x max_batch, staging budget that many packets' bytes (20 each). Each
 * slot holds 16 (max_batch + 1) + 4 max_batch bytes of pinned, coherent host staging and
 * the same of device memory (through the allocator of tang_set_allocator if one is set),
 * until tang_server_destroy. EINVAL on a bad device or configuration (n_streams above 8,
 * max_batch not a power of two of at least 32), EDEVICE without a device.
 */
int tang_server_create(int device, const tang_server_cfg_t* cfg, tang_server_t** out);
/*
 * Register a ruleset (same device); *tag identifies it in submits. May be called while
 * the server runs. The ruleset stays the caller's: an update or model load on it must
 * not overlap its outstanding requests (wait for them first); later batches capture
 * their graphs again.
 */
int tang_server_add_ruleset(tang_server_t* srv, tang_ruleset_t* rs, uint32_t* tag);
/*
 * Record the graphs of every batch size class on every stream slot for ruleset `tag`
 * now, and launch each once on an empty batch, so that its requests do not pay for graph
 * captures or first launches (otherwise each (size class, slot) pair is captured by its
 * first batch). The loop does it while no request is
 * pending and no batch is on the GPU; the call blocks until it is done. The same rule
 * as for requests holds: no update or model load on the ruleset may overlap it. A later
 * update or model load makes batches capture again. EINVAL on a bad tag, EBUSY if the
 * server stops first.
 */
int tang_server_prepare(tang_server_t* srv, uint32_t tag);
/*
 * Submit n host headers for ruleset `tag`; results go to host array out[n] when the
 * request completes. hdr and out must stay valid until then. The serving loop's threads
 * write out: a buffer whose pages were already touched (reused, or written once) keeps
 * first-touch page faults out of the loop. EBUSY if the request can
 * never be admitted (larger than the limits), EINVAL on a bad tag.
 */
int tang_server_submit(tang_server_t* srv, uint32_t tag, const tang_header_t* hdr, size_t n,
                       uint32_t* out, tang_req_t** req);
/* Wait up to timeout_us (< 0: forever). 0 when done, ETIMEOUT otherwise. */
int tang_server_wait(tang_req_t* req, int64_t timeout_us);
/* 1 if done, 0 if not. */
int tang_server_poll(const tang_req_t* req);
/* Timestamps in ns on the host steady clock: submitted, admitted, completed. */
int tang_server_req_times(const tang_req_t* req, uint64_t* submit_ns, uint64_t* admit_ns,
                          uint64_t* done_ns);
/* Frees the handle; a request still running completes (hdr and out must stay valid). */
void tang_server_req_free(tang_req_t* req);
/*
 * Drains pending work, stops the loop, frees the server (not the rulesets). No other
 * call on the same server may be in progress or follow (request handles stay valid:
 * wait, poll, times and free work on them after the server is gone).
 */
int tang_server_destroy(tang_server_t* srv);

#ifdef __cplusplus
}
#endif
#endif /* TANG_H */
