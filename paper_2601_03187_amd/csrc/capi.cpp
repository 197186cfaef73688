// C ABI entry points (include/tang.h): argument checks, error codes, and the calls
// into the host tuple space and the kernels. No C++ exception crosses this boundary.
#include <algorithm>
#include <mutex>
#include <new>
#include <unordered_map>

#include "tang_internal.hpp"

namespace tang {

static thread_local std::string g_err;

// The caller's allocator (tang_set_allocator) and, per block it provided, the free
// callback to return it through.
namespace {
struct Allocator {
    tang_alloc_fn alloc = nullptr;
    tang_free_fn free = nullptr;
    void* ctx = nullptr;
};
struct Owner {
    tang_free_fn free;
    void* ctx;
    int device;
};
std::mutex g_alloc_mu;
Allocator g_alloc;
std::unordered_map<void*, Owner> g_owned;
}  // namespace

hipError_t dev_alloc(void** p, size_t bytes) {
    *p = nullptr;
    Allocator a;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        a = g_alloc;
    }
    if (!a.alloc) return hipMalloc(p, bytes);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    void* q = a.alloc(bytes, dev, a.ctx);
    if (!q) return hipErrorOutOfMemory;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        g_owned[q] = Owner{a.free, a.ctx, dev};
    }
    *p = q;
    // A pool may hand out a block that work still queued on one of its streams uses (a
    // caching allocator recycles a block once it is freed in that stream's order). The
    // library writes the block on streams the pool knows nothing about, so the device
    // must have finished that work first.
    e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        *p = nullptr;
        (void)dev_release(q);
    }
    return e;
}

hipError_t dev_release(void* p) {
    if (!p) return hipSuccess;
    Owner o{nullptr, nullptr, 0};
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        auto it = g_owned.find(p);
        if (it != g_owned.end()) {
            o = it->second;
            g_owned.erase(it);
        }
    }
    if (!o.free) return hipFree(p);
    // hipFree waits for the device's work; so does a release through the caller's
    // allocator, since the block may still be read by kernels in flight on the
    // library's own streams, which the caller's allocator knows nothing about
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != o.device) e = hipSetDevice(o.device);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (cur != o.device) (void)hipSetDevice(cur);
    o.free(p, o.device, o.ctx);
    return e;
}

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return TANG_EDEVICE;
}

// A ruleset whose last update could not be applied on the device refuses every call that
// reads or changes its device state.
static int refuse_failed() {
    return fail(TANG_EDEVICE, "an earlier update of this ruleset failed on the device; destroy "
                              "it and rebuild from tang_ruleset_export");
}

}  // namespace tang

using namespace tang;

size_t tang_ruleset_s::device_bytes() const {
    if (device == TANG_HOST_ONLY) return 0;
    return slots.size() * sizeof(Slot) + filter.size() * sizeof(uint32_t) +
           (size_t)rec_cap * sizeof(Rec) + (nw > 1 ? (size_t)rec_cap * nw * 4 : 0) +
           sizeof(TupleTable) +
           kStatCopies * sizeof(StatsDev) + model.bytes;
}

#define TANG_GUARD_BEGIN try {
#define TANG_GUARD_END                                                   \
    }                                                                    \
    catch (const std::bad_alloc&) {                                      \
        return fail(TANG_ENOMEM, "host allocation failed");              \
    }                                                                    \
    catch (const std::exception& ex) {                                   \
        return fail(TANG_EINVAL, std::string("internal error: ") + ex.what()); \
    }                                                                    \
    catch (...) {                                                        \
        return fail(TANG_EINVAL, "internal error");                      \
    }

static void free_device(tang_ruleset_t* rs) {
    if (rs->device == TANG_HOST_ONLY) return;
    (void)hipSetDevice(rs->device);
    model_free(rs->model);
    if (rs->d_slots) (void)dev_release(rs->d_slots);
    if (rs->d_filter) (void)dev_release(rs->d_filter);
    rs->d_filter = nullptr;
    if (rs->d_recs) (void)dev_release(rs->d_recs);
    if (rs->d_cmask) (void)dev_release(rs->d_cmask);
    rs->d_cmask = nullptr;
    if (rs->d_tt) (void)dev_release(rs->d_tt);
    if (rs->d_stats) (void)dev_release(rs->d_stats);
    for (hipEvent_t e : rs->pipe_events) (void)hipEventDestroy(e);
    rs->pipe_events.clear();
    if (rs->pipe_stream) (void)hipStreamDestroy(rs->pipe_stream);
    rs->pipe_stream = nullptr;
    rs->d_slots = nullptr;
    rs->d_recs = nullptr;
    rs->d_tt = nullptr;
    rs->d_stats = nullptr;
}

extern "C" {

int tang_set_allocator(tang_alloc_fn alloc, tang_free_fn free_fn, void* ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail(TANG_EINVAL, "set both allocator callbacks, or neither");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc = Allocator{alloc, free_fn, alloc ? ctx : nullptr};
    return TANG_OK;
}

const char* tang_last_error(void) { return tang::g_err.c_str(); }

int tang_ruleset_create(int device, const tang_rule_t* rules, size_t n, tang_ruleset_t** out) {
    TANG_GUARD_BEGIN
    if (!out) return fail(TANG_EINVAL, "out is NULL");
    *out = nullptr;
    if (device != TANG_HOST_ONLY) {
        int count = 0;
        hipError_t e = hipGetDeviceCount(&count);
        if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
        if (count == 0) return fail(TANG_EDEVICE, "no HIP device available");
        if (device < 0 || device >= count) return fail(TANG_EINVAL, "bad device ordinal");
    }
    std::unique_ptr<tang_ruleset_t> rs(new tang_ruleset_t());
    rs->device = device;
    int rc = build_host(rs.get(), rules, n);
    if (rc) return rc;
    if (device != TANG_HOST_ONLY) {
        rc = upload_all(rs.get());
        if (rc) {
            free_device(rs.get());
            return rc;
        }
    }
    *out = rs.release();
    return TANG_OK;
    TANG_GUARD_END
}

void tang_ruleset_destroy(tang_ruleset_t* rs) {
    if (!rs) return;
    free_device(rs);
    delete rs;
}

uint32_t tang_ruleset_num_tuples(const tang_ruleset_t* rs) {
    return rs ? (uint32_t)rs->sigs.size() : 0;
}

int tang_ruleset_tuple(const tang_ruleset_t* rs, uint32_t t, uint8_t* sip_len, uint8_t* dip_len) {
    if (!rs || !sip_len || !dip_len) return fail(TANG_EINVAL, "NULL argument");
    if (t >= rs->sigs.size()) return fail(TANG_EINVAL, "tuple index out of range");
    *sip_len = rs->sigs[t].first;
    *dip_len = rs->sigs[t].second;
    return TANG_OK;
}

size_t tang_ruleset_num_rules(const tang_ruleset_t* rs) { return rs ? rs->n_live : 0; }

int tang_ruleset_rule_tuple(const tang_ruleset_t* rs, uint32_t id, uint32_t* tuple) {
    TANG_GUARD_BEGIN
    if (!rs || !tuple) return fail(TANG_EINVAL, "NULL argument");
    auto it = rs->id2h.find(id);
    if (it == rs->id2h.end()) return fail(TANG_ENOTFOUND, "rule id is not live");
    *tuple = rs->rules[it->second].tuple;
    return TANG_OK;
    TANG_GUARD_END
}

int tang_ruleset_conflict_mask_words(tang_ruleset_t* rs, uint32_t id, uint32_t* words,
                                     uint32_t n_words) {
    TANG_GUARD_BEGIN
    if (!rs || (n_words && !words)) return fail(TANG_EINVAL, "NULL argument");
    if (rs->device == TANG_HOST_ONLY) return fail(TANG_EINVAL, "host-only ruleset has no masks");
    if (rs->failed) return refuse_failed();
    auto it = rs->id2h.find(id);
    if (it == rs->id2h.end()) return fail(TANG_ENOTFOUND, "rule id is not live");
    TANG_HIP(hipSetDevice(rs->device));
    const uint32_t pos = rs->rules[it->second].pos;
    Rec r;
    TANG_HIP(hipMemcpy(&r, rs->d_recs + pos, sizeof r, hipMemcpyDeviceToHost));
    if (r.id != id) return fail(TANG_EINVAL, "record/handle mismatch");
    uint32_t row[kMaxWords] = {r.cmask};
    if (rs->nw > 1)
        TANG_HIP(hipMemcpy(row, rs->d_cmask + (size_t)pos * rs->nw, rs->nw * sizeof(uint32_t),
                           hipMemcpyDeviceToHost));
    for (uint32_t w = 0; w < n_words; ++w) words[w] = w < rs->nw ? row[w] : 0u;
    return TANG_OK;
    TANG_GUARD_END
}

int tang_ruleset_conflict_mask(tang_ruleset_t* rs, uint32_t id, uint32_t* mask) {
    if (!mask) return fail(TANG_EINVAL, "NULL argument");
    return tang_ruleset_conflict_mask_words(rs, id, mask, 1);
}

int tang_ruleset_coarse_rules(const tang_ruleset_t* rs, size_t* count) {
    if (!rs || !count) return fail(TANG_EINVAL, "NULL argument");
    *count = rs->n_coarse;
    return TANG_OK;
}

int tang_ruleset_export(const tang_ruleset_t* rs, tang_rule_t* out, size_t cap, size_t* n) {
    TANG_GUARD_BEGIN
    if (!rs || !n) return fail(TANG_EINVAL, "NULL argument");
    *n = rs->n_live;
    if (!out) return TANG_OK;
    if (cap < rs->n_live) return fail(TANG_EINVAL, "export buffer holds fewer than the live rules");
    std::vector<const tang_rule_t*> live;
    live.reserve(rs->n_live);
    for (const auto& hr : rs->rules)
        if (hr.live) live.push_back(&hr.r);
    std::sort(live.begin(), live.end(), [](const tang_rule_t* a, const tang_rule_t* b) {
        return a->priority < b->priority || (a->priority == b->priority && a->id < b->id);
    });
    for (size_t i = 0; i < live.size(); ++i) out[i] = *live[i];
    return TANG_OK;
    TANG_GUARD_END
}

int tang_ruleset_device_bytes(const tang_ruleset_t* rs, size_t* bytes) {
    if (!rs || !bytes) return fail(TANG_EINVAL, "NULL argument");
    *bytes = rs->device_bytes();
    return TANG_OK;
}

int tang_ruleset_set_stream(tang_ruleset_t* rs, void* stream) {
    if (!rs) return fail(TANG_EINVAL, "NULL ruleset");
    rs->upd_stream = (hipStream_t)stream;
    return TANG_OK;
}

int tang_model_load(tang_ruleset_t* rs, const tang_mlp_desc_t* desc, const float* const* W,
                    const float* const* b, tang_precision_t precision, const float* act_scales) {
    TANG_GUARD_BEGIN
    if (!rs) return fail(TANG_EINVAL, "NULL ruleset");
    if (rs->device == TANG_HOST_ONLY) return fail(TANG_EINVAL, "host-only ruleset cannot hold a model");
    if (rs->failed) return refuse_failed();
    TANG_HIP(hipSetDevice(rs->device));
    TANG_HIP(hipDeviceSynchronize());  // no classify may still read the old weights
    return model_prepare(rs, desc, W, b, precision, act_scales);
    TANG_GUARD_END
}

int tang_model_load_resnet(tang_ruleset_t* rs, const tang_resnet_desc_t* desc, const float* const* W,
                           const float* const* b, tang_precision_t precision) {
    TANG_GUARD_BEGIN
    if (!rs) return fail(TANG_EINVAL, "NULL ruleset");
    if (rs->device == TANG_HOST_ONLY) return fail(TANG_EINVAL, "host-only ruleset cannot hold a model");
    if (rs->failed) return refuse_failed();
    TANG_HIP(hipSetDevice(rs->device));
    TANG_HIP(hipDeviceSynchronize());  // no classify may still read the old weights
    return resnet_prepare(rs, desc, W, b, precision);
    TANG_GUARD_END
}

int tang_model_unload(tang_ruleset_t* rs) {
    if (!rs) return fail(TANG_EINVAL, "NULL ruleset");
    if (rs->device != TANG_HOST_ONLY) {
        TANG_HIP(hipSetDevice(rs->device));
        TANG_HIP(hipDeviceSynchronize());
    }
    model_free(rs->model);
    rs->version++;
    return TANG_OK;
}

}  // extern "C"

static int check_classify(const tang_ruleset_t* rs, const void* hdr, const void* out, size_t n) {
    if (!rs) return fail(TANG_EINVAL, "NULL ruleset");
    if (rs->device == TANG_HOST_ONLY) return fail(TANG_EINVAL, "host-only ruleset cannot classify");
    if (rs->failed) return refuse_failed();
    if (n && (!hdr || !out)) return fail(TANG_EINVAL, "NULL buffer");
    if (((uintptr_t)hdr & 15u) != 0) return fail(TANG_EINVAL, "headers must be 16-byte aligned");
    if (((uintptr_t)out & 3u) != 0) return fail(TANG_EINVAL, "rule_id buffer must be 4-byte aligned");
    return TANG_OK;
}

static int run_search(tang_ruleset_t* rs, const tang_header_t* d_hdr, uint32_t* d_io, size_t n,
                      hipStream_t s, tang_stats_t* stats, const uint32_t* d_live = nullptr) {
    std::unique_lock<std::mutex> lk(rs->stats_mu, std::defer_lock);
    if (stats) {
        lk.lock();
        TANG_HIP(hipMemsetAsync(rs->d_stats, 0, kStatCopies * sizeof(StatsDev), s));
    }
    const int kcand = rs->model.loaded ? rs->model.topk : 0;
    TANG_HIP(launch_classify(rs, d_hdr, d_io, n, kcand, s, stats != nullptr, d_live));
    if (stats) {
        StatsDev part[kStatCopies], h;
        std::memset(&h, 0, sizeof h);
        TANG_HIP(hipMemcpyAsync(part, rs->d_stats, sizeof part, hipMemcpyDeviceToHost, s));
        TANG_HIP(hipStreamSynchronize(s));
        for (const StatsDev& p : part) {
            h.packets += p.packets; h.probes += p.probes; h.slots += p.slots;
            h.records += p.records; h.top1 += p.top1; h.fallbacks += p.fallbacks;
            h.nomatch += p.nomatch; h.filters += p.filters; h.steps += p.steps;
            h.rounds += p.rounds;
        }
        stats->packets = h.packets;
        stats->probes = h.probes;
        stats->slots = h.slots;
        stats->records = h.records;
        stats->top1_hits = h.top1;
        stats->fallbacks = h.fallbacks;
        stats->no_match = h.nomatch;
        stats->filter_checks = h.filters;
        stats->wave_steps = h.steps;
        stats->wave_rounds = h.rounds;
    }
    return TANG_OK;
}

// Large batches with a model: chunk k's model runs on the caller's stream while chunk
// k-1's search runs on the ruleset's own stream, so the MFMA-bound and the latency-bound
// kernels overlap (and a chunk's headers are still cached when its search reads them).
// The caller's stream waits for the last search, so the call completes in stream order.
// If another thread is enqueueing a chunked call on the same ruleset, this call takes
// the plain path instead of waiting for the lock.
static int classify_chunked(tang_ruleset_t* rs, const tang_header_t* d_hdr, uint32_t* out,
                            size_t n, hipStream_t s, bool* done) {
    *done = false;
    std::unique_lock<std::mutex> lk(rs->pipe_mu, std::try_to_lock);
    if (!lk.owns_lock()) return TANG_OK;
    if (!rs->pipe_stream) TANG_HIP(hipStreamCreateWithFlags(&rs->pipe_stream, hipStreamNonBlocking));
    // A half chunk first and last (the first chunk's predictor and the last chunk's search
    // run with nothing beside them), the rest in equal parts of at most kPipeChunk;
    // n >= 2 kPipeChunk here.
    const size_t E = kPipeChunk / 2, M = n - 2 * E;
    const size_t q = (M + kPipeChunk - 1) / kPipeChunk, part = (M + q - 1) / q;
    std::vector<size_t> sz{E};
    for (size_t left = M; left > 0; left -= std::min(part, left)) sz.push_back(std::min(part, left));
    sz.push_back(E);
    const size_t K = sz.size();
    while (rs->pipe_events.size() < K + 1) {
        hipEvent_t e = nullptr;
        TANG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        rs->pipe_events.push_back(e);
    }
    const int kcand = rs->model.topk;
    size_t base = 0;
    for (size_t k = 0; k < K; base += sz[k], ++k) {
        const size_t m = sz[k];
        TANG_HIP(launch_mlp(rs, d_hdr + base, m, out + base, nullptr, nullptr, s, true));
        TANG_HIP(hipEventRecord(rs->pipe_events[k], s));
        TANG_HIP(hipStreamWaitEvent(rs->pipe_stream, rs->pipe_events[k], 0));
        TANG_HIP(launch_classify(rs, d_hdr + base, out + base, m, kcand, rs->pipe_stream, false));
    }
    TANG_HIP(hipEventRecord(rs->pipe_events[K], rs->pipe_stream));
    TANG_HIP(hipStreamWaitEvent(s, rs->pipe_events[K], 0));
    *done = true;
    return TANG_OK;
}

namespace tang {
int classify_async(tang_ruleset_t* rs, const tang_header_t* d_hdr, uint32_t* d_rule_id, size_t n,
                   hipStream_t s, tang_stats_t* stats, bool allow_chunks, const uint32_t* d_live) {
    int rc = check_classify(rs, d_hdr, d_rule_id, n);
    if (rc) return rc;
    if (d_live && (stats || allow_chunks || rs->model.kind != 0))
        return fail(TANG_EINVAL, "a live-count launch takes no stats, chunks or residual model");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n == 0) return TANG_OK;
    TANG_HIP(hipSetDevice(rs->device));
    // (an FP32 model's MLP takes several times the search: nothing to overlap)
    if (allow_chunks && rs->model.loaded && rs->model.prec != TANG_FP32 && !stats &&
        n >= 2 * kPipeChunk) {
        bool done = false;
        rc = classify_chunked(rs, d_hdr, d_rule_id, n, s, &done);
        if (rc || done) return rc;
    }
    if (rs->model.loaded) TANG_HIP(launch_mlp(rs, d_hdr, n, d_rule_id, nullptr, nullptr, s, false, d_live));
    return run_search(rs, d_hdr, d_rule_id, n, s, stats, d_live);
}
}  // namespace tang

extern "C" {

int tang_classify(tang_ruleset_t* rs, const tang_header_t* d_hdr, uint32_t* d_rule_id, size_t n,
                  void* stream, tang_stats_t* stats) {
    TANG_GUARD_BEGIN
    return classify_async(rs, d_hdr, d_rule_id, n, (hipStream_t)stream, stats, true);
    TANG_GUARD_END
}

int tang_predict(tang_ruleset_t* rs, const tang_header_t* d_hdr, uint32_t* d_io, size_t n,
                 void* stream) {
    TANG_GUARD_BEGIN
    int rc = check_classify(rs, d_hdr, d_io, n);
    if (rc) return rc;
    if (!rs->model.loaded) return fail(TANG_EINVAL, "no model loaded");
    if (n == 0) return TANG_OK;
    TANG_HIP(hipSetDevice(rs->device));
    TANG_HIP(launch_mlp(rs, d_hdr, n, d_io, nullptr, nullptr, (hipStream_t)stream));
    return TANG_OK;
    TANG_GUARD_END
}

int tang_search(tang_ruleset_t* rs, const tang_header_t* d_hdr, uint32_t* d_io, size_t n,
                void* stream, tang_stats_t* stats) {
    TANG_GUARD_BEGIN
    int rc = check_classify(rs, d_hdr, d_io, n);
    if (rc) return rc;
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n == 0) return TANG_OK;
    TANG_HIP(hipSetDevice(rs->device));
    return run_search(rs, d_hdr, d_io, n, (hipStream_t)stream, stats);
    TANG_GUARD_END
}

int tang_search_host(const tang_ruleset_t* rs, const tang_header_t* hdr, const uint32_t* cand,
                     uint32_t* rule_id, size_t n, uint32_t kcand, uint32_t threads, int exact,
                     tang_stats_t* stats) {
    TANG_GUARD_BEGIN
    if (!rs) return fail(TANG_EINVAL, "NULL ruleset");
    if (kcand > (rs->sigs.size() > 256 ? 2u : (uint32_t)TANG_MAX_TOPK))
        return fail(TANG_EINVAL, "kcand must be in 0..4 (0..2 above 256 tuples)");
    if (n && (!hdr || !rule_id || (kcand && !cand))) return fail(TANG_EINVAL, "NULL buffer");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n == 0) return TANG_OK;
    return search_host(rs, hdr, cand, rule_id, n, kcand, threads, exact != 0, stats);
    TANG_GUARD_END
}

int tang_classify_host(tang_ruleset_t* rs, const tang_header_t* hdr, uint32_t* rule_id, size_t n,
                       tang_stats_t* stats) {
    TANG_GUARD_BEGIN
    if (!rs) return fail(TANG_EINVAL, "NULL ruleset");
    if (rs->device == TANG_HOST_ONLY) return fail(TANG_EINVAL, "host-only ruleset cannot classify");
    if (rs->failed) return refuse_failed();
    if (n && (!hdr || !rule_id)) return fail(TANG_EINVAL, "NULL buffer");
    if (n > SIZE_MAX / sizeof(tang_header_t)) return fail(TANG_EINVAL, "n too large");
    if (stats) std::memset(stats, 0, sizeof *stats);
    if (n == 0) return TANG_OK;
    TANG_HIP(hipSetDevice(rs->device));
    tang_header_t* dh = nullptr;
    uint32_t* dout = nullptr;
    TANG_HIP(dev_alloc(&dh, n * sizeof(tang_header_t)));
    hipError_t e = dev_alloc(&dout, n * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemcpy(dh, hdr, n * sizeof(tang_header_t), hipMemcpyHostToDevice);
    int rc = TANG_OK;
    if (e == hipSuccess) {
        rc = tang_classify(rs, dh, dout, n, nullptr, stats);
        if (rc == TANG_OK) e = hipMemcpy(rule_id, dout, n * sizeof(uint32_t), hipMemcpyDeviceToHost);
    }
    (void)dev_release(dh);
    if (dout) (void)dev_release(dout);
    if (e != hipSuccess) return hip_fail(e, "tang_classify_host");
    return rc;
    TANG_GUARD_END
}

int tang_mlp_forward(tang_ruleset_t* rs, const tang_header_t* d_hdr, size_t n, float* d_logits,
                     uint16_t* d_cand, void* stream) {
    TANG_GUARD_BEGIN
    if (!rs) return fail(TANG_EINVAL, "NULL ruleset");
    if (rs->device == TANG_HOST_ONLY || !rs->model.loaded) return fail(TANG_EINVAL, "no model loaded");
    if (rs->failed) return refuse_failed();
    if (n && !d_hdr) return fail(TANG_EINVAL, "NULL headers");
    if (((uintptr_t)d_hdr & 15u) != 0) return fail(TANG_EINVAL, "headers must be 16-byte aligned");
    if (n == 0) return TANG_OK;
    TANG_HIP(hipSetDevice(rs->device));
    TANG_HIP(launch_mlp(rs, d_hdr, n, nullptr, d_logits, d_cand, (hipStream_t)stream));
    return TANG_OK;
    TANG_GUARD_END
}

int tang_insert(tang_ruleset_t* rs, const tang_rule_t* rules, size_t n) {
    TANG_GUARD_BEGIN
    if (!rs) return fail(TANG_EINVAL, "NULL ruleset");
    if (rs->failed) return refuse_failed();
    return apply_insert(rs, rules, n);
    TANG_GUARD_END
}

int tang_delete(tang_ruleset_t* rs, const uint32_t* ids, size_t n) {
    TANG_GUARD_BEGIN
    if (!rs) return fail(TANG_EINVAL, "NULL ruleset");
    if (rs->failed) return refuse_failed();
    return apply_delete(rs, ids, n);
    TANG_GUARD_END
}

}  // extern "C"
