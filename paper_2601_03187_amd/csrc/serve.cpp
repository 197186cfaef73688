// Serving loop: continuous batching of classify requests over device-resident rulesets.
//
// One persistent host thread owns S stream slots. Each slot has pinned host staging
// and device buffers for one batch. While a slot is free and requests are pending, the
// loop takes the oldest pending request, packs further pending requests of the same
// ruleset behind it (arrival order, up to the batch limit), admits them if the packets
// and staging bytes in flight stay within the configured limits, writes their headers
// into the slot's pinned staging, replays the HIP graph captured for (ruleset, batch size
// class, slot) and records an event. Completed slots hand results to their requests.
// Up to 65,536 headers the graph moves the batch itself: a first kernel pulls the
// headers from the pinned staging into device memory, a last one pushes the rule ids
// back, so that a batch costs one graph launch and no runtime copy (asynchronous runtime
// copies have been seen to hold the calling thread for 6-11 ms now and then, which
// stalled admission for every slot when the loop issued them). Larger batches go through
// the copy engines, faster than kernel reads of host memory, issued around the graph by
// the slot's own thread (SlotIssuer), so that a held call delays only that slot.
// A graph is recorded for the largest batch of its size class (a power of two); the
// batch's real header count travels with its headers (the first 16 bytes of the slot's
// staging) and the kernels read it from there, so a batch
// costs the work of its own headers, not of its class. On request
// (tang_server_prepare) the loop records the graphs of every size class on every slot
// of a ruleset while no request is pending and no batch is on the GPU (yielding to
// requests as they arrive) and launches each once on an empty batch, so that requests
// pay neither for graph captures nor for first launches.
// Requests that arrive while others are on the GPU are admitted as slots and budget
// free up, so batches of different requests and rulesets overlap on the device. The host
// copies of a large batch (its headers into the staging, its rule ids back out) are spread
// over the loop thread and three helper threads.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

#include "tang_internal.hpp"

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct ReqState {
    uint32_t tag = 0;
    const tang_header_t* hdr = nullptr;
    size_t n = 0;
    uint32_t* out = nullptr;
    uint64_t t_submit = 0, t_admit = 0, t_done = 0;
    int status = TANG_OK;
    bool done = false;
    std::mutex mu;
    std::condition_variable cv;
};

struct StreamSlot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    // staging of max_batch + 1 headers: element 0 carries the live count in its first
    // word, the batch's headers follow; the pinned host halves are coherent host memory
    // that the staging kernels read and write through their device addresses (dh_*)
    tang_header_t* h_buf = nullptr;  // pinned
    uint32_t* h_out = nullptr;       // pinned
    const tang_header_t* dh_buf = nullptr;
    uint32_t* dh_out = nullptr;
    tang_header_t* d_buf = nullptr;
    uint32_t* d_out = nullptr;
    tang_header_t* h_hdr() const { return h_buf + 1; }
    tang_header_t* d_hdr() const { return d_buf + 1; }
    const uint32_t* d_live() const { return reinterpret_cast<const uint32_t*>(d_buf); }
    bool busy = false;
    bool issued_by_slot = false;   // the batch was posted to the slot's issuer thread
    size_t total = 0;
    std::vector<std::shared_ptr<ReqState>> reqs;
    std::vector<size_t> offs;
};

struct GraphEntry {
    uint64_t version = ~0ull;
    hipGraphExec_t exec = nullptr;
};

// Host copies of a batch (headers into the pinned staging, rule ids out of it) spread over
// the loop thread and a few helper threads: one thread's memcpy moves a large batch
// several times slower than the GPU classifies it. run() returns once every chunk is
// copied and every helper has let go of the chunk list.
struct CopyChunk {
    void* dst;
    const void* src;
    size_t n;
};
static constexpr size_t kChunkBytes = 256u << 10;
// batches below this many headers (single requests included: they are at most 65,536
// headers in the serving workload) copy on the loop thread alone, without waking helpers
static constexpr size_t kPoolMinHeaders = 131072;
static constexpr unsigned kCopyHelpers = 3;

class CopyPool {
  public:
    explicit CopyPool(unsigned helpers) {
        for (unsigned k = 0; k < helpers; ++k) th_.emplace_back([this] { work(); });
    }
    ~CopyPool() {
        {
            std::lock_guard<std::mutex> g(mu_);
            stop_ = true;
        }
        cv_.notify_all();
        for (auto& t : th_) t.join();
    }
    // Appends the copy of n bytes, cut into chunks.
    static void add(std::vector<CopyChunk>& c, void* dst, const void* src, size_t n) {
        for (size_t off = 0; off < n; off += kChunkBytes)
            c.push_back(CopyChunk{static_cast<char*>(dst) + off, static_cast<const char*>(src) + off,
                                  std::min(kChunkBytes, n - off)});
    }
    void run(const std::vector<CopyChunk>& c, bool spread) {
        if (th_.empty() || !spread) {
            for (const auto& x : c) std::memcpy(x.dst, x.src, x.n);
            return;
        }
        {
            std::lock_guard<std::mutex> g(mu_);
            job_ = &c;
            next_.store(0);
            busy_ = th_.size();
            ++gen_;
        }
        cv_.notify_all();
        grab(c);
        std::unique_lock<std::mutex> lk(mu_);
        done_cv_.wait(lk, [&] { return busy_ == 0; });
        job_ = nullptr;
    }

  private:
    void grab(const std::vector<CopyChunk>& c) {
        for (size_t k; (k = next_.fetch_add(1)) < c.size();) std::memcpy(c[k].dst, c[k].src, c[k].n);
    }
    void work() {
        uint64_t seen = 0;
        for (;;) {
            const std::vector<CopyChunk>* j = nullptr;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
                if (stop_) return;
                seen = gen_;
                j = job_;
            }
            grab(*j);
            {
                std::lock_guard<std::mutex> g(mu_);
                if (--busy_ == 0) done_cv_.notify_all();
            }
        }
    }
    std::vector<std::thread> th_;
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    const std::vector<CopyChunk>* job_ = nullptr;
    std::atomic<size_t> next_{0};
    size_t busy_ = 0;
    uint64_t gen_ = 0;
    bool stop_ = false;
};

// Batches of the large size classes move through the copy engines (hipMemcpyAsync: about
// 1.3x the rate of the staging kernels' reads of host memory). A runtime copy call has been
// seen to hold its calling thread for 6-11 ms now and then, so these batches are issued by
// the slot's own thread and a held call never blocks the loop thread itself (other HIP
// work can still wait behind it inside the runtime: once, a whole burst came out about
// 8 ms late).
// The loop posts a batch (its staging is written, its graph recorded) and, once issued()
// turns true, polls the slot's event as for any batch.
class SlotIssuer {
  public:
    SlotIssuer(int device, StreamSlot* s) : s_(s), th_([this, device] { work(device); }) {}
    ~SlotIssuer() {
        {
            std::lock_guard<std::mutex> g(mu_);
            quit_ = true;
        }
        cv_.notify_all();
        th_.join();
    }
    void post(hipGraphExec_t exec, size_t total) {
        issued_.store(false, std::memory_order_relaxed);
        {
            std::lock_guard<std::mutex> g(mu_);
            exec_ = exec;
            total_ = total;
            job_ = true;
        }
        cv_.notify_one();
    }
    bool issued() const { return issued_.load(std::memory_order_acquire); }
    int status() const { return status_; }   // valid once issued()

  private:
    void work(int device) {
        (void)hipSetDevice(device);
        for (;;) {
            hipGraphExec_t exec;
            size_t total;
            {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] { return quit_ || job_; });
                if (quit_) return;
                job_ = false;
                exec = exec_;
                total = total_;
            }
            StreamSlot& s = *s_;
            hipError_t e = hipMemcpyAsync(s.d_buf, s.h_buf, (total + 1) * sizeof(tang_header_t),
                                          hipMemcpyHostToDevice, s.stream);
            if (e == hipSuccess) e = hipGraphLaunch(exec, s.stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(s.h_out, s.d_out, total * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                   s.stream);
            if (e == hipSuccess) e = hipEventRecord(s.ev, s.stream);
            status_ = e == hipSuccess ? TANG_OK : TANG_EDEVICE;
            issued_.store(true, std::memory_order_release);
        }
    }
    StreamSlot* s_;
    std::mutex mu_;
    std::condition_variable cv_;
    bool job_ = false, quit_ = false;
    hipGraphExec_t exec_ = nullptr;
    size_t total_ = 0;
    int status_ = TANG_OK;
    std::atomic<bool> issued_{true};
    std::thread th_;
};
// size classes that use SlotIssuer: batches of more than 65,536 headers, which only form
// when requests queue up and merge
static constexpr uint64_t kCopyEngineClass = 1u << 17;

constexpr uint32_t kStageThreads = 256;
constexpr uint32_t kInPerThread = 4;    // headers per thread of k_stage_in
constexpr uint32_t kOutPerThread = 4;   // rule ids per thread of k_stage_out

// Pulls a batch from pinned host staging into device memory: element 0 (the live count
// in its first word) and then the live headers, kInPerThread 16-byte headers per thread
// (all loads issued before the stores: reads of host memory are long round trips);
// threads past the live count (or the launch's capacity) do nothing.
__global__ void __launch_bounds__(kStageThreads)
k_stage_in(const uint4* __restrict__ h_buf, uint4* __restrict__ d_buf, uint32_t cap) {
    const uint4 head = h_buf[0];
    const uint32_t live = min(head.x, cap);
    const uint32_t i0 = blockIdx.x * kStageThreads * kInPerThread + threadIdx.x;
    if (i0 == 0) d_buf[0] = head;
    uint4 v[kInPerThread];
#pragma unroll
    for (uint32_t k = 0; k < kInPerThread; ++k) {
        const uint32_t i = i0 + k * kStageThreads;
        if (i < live) v[k] = h_buf[1 + i];
    }
#pragma unroll
    for (uint32_t k = 0; k < kInPerThread; ++k) {
        const uint32_t i = i0 + k * kStageThreads;
        if (i < live) d_buf[1 + i] = v[k];
    }
}

// Pushes the batch's rule ids to pinned host memory, kOutPerThread (4) per thread (one
// 16-byte store where all four are live); the live count is the one k_stage_in wrote.
__global__ void __launch_bounds__(kStageThreads)
k_stage_out(const uint32_t* __restrict__ d_live, const uint32_t* __restrict__ d_out,
            uint32_t* __restrict__ h_out, uint32_t cap) {
    const uint32_t live = min(d_live[0], cap);
    static_assert(kOutPerThread == 4, "one 16-byte store per thread");
    const uint32_t j = kOutPerThread * (blockIdx.x * kStageThreads + threadIdx.x);
    if (j + kOutPerThread <= live) {
        *reinterpret_cast<uint4*>(h_out + j) = *reinterpret_cast<const uint4*>(d_out + j);
    } else {
        for (uint32_t k = j; k < live; ++k) h_out[k] = d_out[k];
    }
}

}  // namespace

struct tang_req_s {
    std::shared_ptr<ReqState> st;
};

struct tang_server_s {
    int device = 0;
    tang_server_cfg_t cfg{};
    std::vector<tang_ruleset_t*> rulesets;
    std::vector<StreamSlot> slots;
    std::map<std::tuple<uint32_t, uint32_t, uint32_t>, GraphEntry> graphs;  // (tag, class, slot)
    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<ReqState>> pending;
    size_t inflight_pkts = 0, inflight_bytes = 0;
    bool stop = false;
    std::thread th;
    std::vector<char> warmed;
    std::vector<char> prepared;   // 0 not asked, 1 asked, 2 every (class, slot) graph recorded
    std::condition_variable prepared_cv;
    std::unique_ptr<CopyPool> copies;   // used by the loop thread only
    std::vector<CopyChunk> chunks;
    std::vector<std::unique_ptr<SlotIssuer>> issuers;   // one per slot

    void loop();
    void finish(StreamSlot& s, int status);
    int launch(uint32_t slot_idx, uint32_t tag, tang_ruleset_t* rs, bool warm,
               std::vector<std::shared_ptr<ReqState>>& batch, size_t total);
    int graph_for(uint32_t tag, tang_ruleset_t* rs, uint32_t cls, uint32_t slot_idx,
                  hipGraphExec_t* out);
    bool prepare(uint32_t tag, tang_ruleset_t* rs, bool warm);
    int run_batch(tang_ruleset_t* rs, StreamSlot& s, size_t cap, bool live_count, bool staged = true);
};

using namespace tang;

static constexpr size_t kPktBytes = sizeof(tang_header_t) + sizeof(uint32_t);

// Only the loop thread calls launch and graph_for; `rulesets` and `warmed` may grow under
// `mu` meanwhile (tang_server_add_ruleset), so the loop reads them under `mu` and passes
// the ruleset and its warm-up flag in.
int tang_server_s::graph_for(uint32_t tag, tang_ruleset_t* rs, uint32_t cls, uint32_t si,
                             hipGraphExec_t* out) {
    GraphEntry& g = graphs[std::make_tuple(tag, cls, si)];
    if (g.exec && g.version == rs->version) {
        *out = g.exec;
        return TANG_OK;
    }
    if (g.exec) {
        (void)hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
    }
    StreamSlot& s = slots[si];
    TANG_HIP(hipStreamBeginCapture(s.stream, hipStreamCaptureModeRelaxed));
    int rc = run_batch(rs, s, cls, true, cls < kCopyEngineClass);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s.stream, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        g.exec = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
    }
    g.version = rs->version;
    *out = g.exec;
    return TANG_OK;
}

// One batch of up to `cap` headers on the slot's stream: the headers in, the
// classification, the rule ids out. With `live_count` the kernels take the batch's size
// from the staging (launches sized for `cap`, as a graph records them); without it `cap`
// is the batch's size.
int tang_server_s::run_batch(tang_ruleset_t* rs, StreamSlot& s, size_t cap, bool live_count,
                             bool staged) {
    // a copy-engine batch's graph is the classification alone (its copies are issued around it)
    if (!staged) return classify_async(rs, s.d_hdr(), s.d_out, cap, s.stream, nullptr, false, s.d_live());
    const uint32_t c = (uint32_t)cap;   // cap <= max_batch, a 32-bit value
    constexpr uint32_t in_blk = kInPerThread * kStageThreads, out_blk = kOutPerThread * kStageThreads;
    hipLaunchKernelGGL(k_stage_in, dim3((c + in_blk - 1) / in_blk), dim3(kStageThreads),
                       0, s.stream, reinterpret_cast<const uint4*>(s.dh_buf),
                       reinterpret_cast<uint4*>(s.d_buf), c);
    TANG_HIP(hipGetLastError());
    int rc = classify_async(rs, s.d_hdr(), s.d_out, cap, s.stream, nullptr, false,
                            live_count ? s.d_live() : nullptr);
    if (rc) return rc;
    hipLaunchKernelGGL(k_stage_out, dim3((c + out_blk - 1) / out_blk),
                       dim3(kStageThreads), 0, s.stream, s.d_live(), s.d_out, s.dh_out, c);
    TANG_HIP(hipGetLastError());
    return TANG_OK;
}

int tang_server_s::launch(uint32_t si, uint32_t tag, tang_ruleset_t* rs, bool warm,
                          std::vector<std::shared_ptr<ReqState>>& batch, size_t total) {
    StreamSlot& s = slots[si];
    s.reqs = batch;
    s.offs.clear();
    s.total = total;
    size_t off = 0;
    chunks.clear();
    for (auto& r : batch) {
        s.offs.push_back(off);
        CopyPool::add(chunks, s.h_hdr() + off, r->hdr, r->n * sizeof(tang_header_t));
        off += r->n;
    }
    copies->run(chunks, total >= kPoolMinHeaders);
    size_t cls = 32;
    while (cls < total) cls <<= 1;
    const uint32_t live = (uint32_t)total;   // total <= max_batch, a 32-bit value
    s.h_buf[0] = tang_header_t{};
    std::memcpy(&s.h_buf[0], &live, sizeof live);
    if (!warm) {  // first use: an eager batch sets up kernel attributes before any capture
        int rc = run_batch(rs, s, total, false);
        if (rc) return rc;
        TANG_HIP(hipStreamSynchronize(s.stream));
    }
    // the residual predictor orders its shared workspace with an event across calls, which
    // a captured graph cannot hold: its batches run eagerly
    if (cfg.use_graphs && rs->model.kind == 0) {
        hipGraphExec_t exec = nullptr;
        int rc = graph_for(tag, rs, (uint32_t)cls, si, &exec);
        if (rc) return rc;
        if (cls >= kCopyEngineClass) {
            issuers[si]->post(exec, total);
            s.issued_by_slot = true;
            s.busy = true;
            return TANG_OK;
        }
        TANG_HIP(hipGraphLaunch(exec, s.stream));
    } else {
        int rc = run_batch(rs, s, total, false);
        if (rc) return rc;
    }
    TANG_HIP(hipEventRecord(s.ev, s.stream));
    s.busy = true;
    return TANG_OK;
}

// Preparation of ruleset `tag` (asked for by tang_server_prepare, run by the loop while
// idle): the eager first call (kernel attributes) if needed, then the graph of every
// size class on every slot. Returns false if it stopped early because a request arrived
// (it resumes at the next idle moment; recorded graphs stay). Failures are left to the
// request path, which reports them.
bool tang_server_s::prepare(uint32_t tag, tang_ruleset_t* rs, bool warm) {
    if (!cfg.use_graphs || rs->model.kind != 0) return true;
    StreamSlot& s0 = slots[0];
    if (!warm) {
        if (classify_async(rs, s0.d_hdr(), s0.d_out, 32, s0.stream, nullptr, false) != TANG_OK) return true;
        if (hipStreamSynchronize(s0.stream) != hipSuccess) return true;
        std::lock_guard<std::mutex> g(mu);
        warmed[tag] = 1;
    }
    // the graphs of a slot, once recorded, are each launched once (a graph's first launch
    // costs more than a replay) with a live count of 0 in the slot's staging, so their
    // kernels return at once; the stream is drained before the loop uses the slot again
    for (uint32_t si = 0; si < slots.size(); ++si) {
        std::vector<hipGraphExec_t> execs;
        for (uint64_t cls = 32; cls <= cfg.max_batch; cls <<= 1) {
            {
                std::lock_guard<std::mutex> g(mu);
                if (!pending.empty() || stop) return false;
            }
            hipGraphExec_t exec = nullptr;
            if (graph_for(tag, rs, (uint32_t)cls, si, &exec) != TANG_OK) return true;
            execs.push_back(exec);
        }
        StreamSlot& s = slots[si];
        s.h_buf[0] = tang_header_t{};
        // the copy-engine classes' graphs read the live count from device memory
        hipError_t e = hipMemcpyAsync(s.d_buf, s.h_buf, sizeof(tang_header_t), hipMemcpyHostToDevice,
                                      s.stream);
        for (size_t k = 0; k < execs.size() && e == hipSuccess; ++k)
            e = hipGraphLaunch(execs[k], s.stream);
        // one full-size copy each way on the slot's stream, so that the copy engines' first
        // use (which can take milliseconds) falls here rather than on a request
        if (e == hipSuccess && cfg.max_batch >= kCopyEngineClass)
            e = hipMemcpyAsync(s.d_buf, s.h_buf, ((size_t)cfg.max_batch + 1) * sizeof(tang_header_t),
                               hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess && cfg.max_batch >= kCopyEngineClass)
            e = hipMemcpyAsync(s.h_out, s.d_out, (size_t)cfg.max_batch * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, s.stream);
        (void)hipStreamSynchronize(s.stream);
        if (e != hipSuccess) return true;
    }
    return true;
}

void tang_server_s::finish(StreamSlot& s, int status) {
    if (status == TANG_OK) {
        chunks.clear();
        for (size_t k = 0; k < s.reqs.size(); ++k)
            CopyPool::add(chunks, s.reqs[k]->out, s.h_out + s.offs[k], s.reqs[k]->n * sizeof(uint32_t));
        copies->run(chunks, s.total >= kPoolMinHeaders);
    }
    const uint64_t t = now_ns();
    for (size_t k = 0; k < s.reqs.size(); ++k) {
        auto& r = s.reqs[k];
        {
            std::lock_guard<std::mutex> g(r->mu);
            r->t_done = t;
            r->status = status;
            r->done = true;
        }
        r->cv.notify_all();
    }
    {
        std::lock_guard<std::mutex> g(mu);
        inflight_pkts -= s.total;
        inflight_bytes -= s.total * kPktBytes;
    }
    s.reqs.clear();
    s.busy = false;
    s.issued_by_slot = false;
    s.total = 0;
}

void tang_server_s::loop() {
    (void)hipSetDevice(device);  // the ordinal was checked at creation
    for (;;) {
        bool progressed = false;
        for (uint32_t si = 0; si < slots.size(); ++si) {
            StreamSlot& s = slots[si];
            if (!s.busy) continue;
            if (s.issued_by_slot) {
                if (!issuers[si]->issued()) continue;   // its event is not recorded yet
                if (issuers[si]->status() != TANG_OK) {
                    finish(s, issuers[si]->status());
                    progressed = true;
                    continue;
                }
            }
            hipError_t q = hipEventQuery(s.ev);
            if (q == hipSuccess) {
                finish(s, TANG_OK);
                progressed = true;
            } else if (q != hipErrorNotReady) {
                finish(s, TANG_EDEVICE);
                progressed = true;
            }
        }
        std::unique_lock<std::mutex> lk(mu);
        bool any_busy = false;
        for (auto& s : slots) any_busy |= s.busy;
        if (stop && pending.empty() && !any_busy) {
            prepared_cv.notify_all();
            break;
        }
        for (uint32_t si = 0; si < slots.size() && !pending.empty(); ++si) {
            if (slots[si].busy) continue;
            // oldest request decides the ruleset; same-ruleset requests behind it join
            const uint32_t tag = pending.front()->tag;
            std::vector<std::shared_ptr<ReqState>> batch;
            size_t total = 0;
            for (auto it = pending.begin(); it != pending.end();) {
                if ((*it)->tag != tag) { ++it; continue; }
                const size_t n = (*it)->n;
                if (total + n > cfg.max_batch) break;
                if (inflight_pkts + total + n > cfg.max_inflight_packets) break;
                if (inflight_bytes + (total + n) * kPktBytes > cfg.mem_budget_bytes) break;
                batch.push_back(*it);
                total += n;
                it = pending.erase(it);
            }
            if (batch.empty()) break;  // not admissible yet: wait for completions
            inflight_pkts += total;
            inflight_bytes += total * kPktBytes;
            const uint64_t t = now_ns();
            for (auto& r : batch) r->t_admit = t;
            tang_ruleset_t* rs = rulesets[tag];
            const bool warm = warmed[tag] != 0;
            lk.unlock();
            int rc = launch(si, tag, rs, warm, batch, total);
            if (rc != TANG_OK) {
                StreamSlot& s = slots[si];
                s.reqs = batch;
                s.total = total;
                s.offs.assign(batch.size(), 0);
                finish(s, rc);
            }
            progressed = true;
            lk.lock();
            if (rc == TANG_OK) warmed[tag] = 1;
        }
        if (!progressed) {
            any_busy = false;
            for (auto& s : slots) any_busy |= s.busy;
            if (any_busy) {
                cv.wait_for(lk, std::chrono::microseconds(20));
            } else if (pending.empty() && !stop) {
                uint32_t tag = 0;
                while (tag < prepared.size() && prepared[tag] != 1) ++tag;
                if (tag < prepared.size()) {
                    tang_ruleset_t* rs = rulesets[tag];
                    const bool warm = warmed[tag] != 0;
                    lk.unlock();
                    const bool done = prepare(tag, rs, warm);
                    lk.lock();
                    if (done) {
                        prepared[tag] = 2;
                        prepared_cv.notify_all();
                    }
                } else {
                    cv.wait_for(lk, std::chrono::milliseconds(50));
                }
            }
        }
    }
}

static void free_server(tang_server_t* srv) {
    srv->issuers.clear();   // joins the issuer threads (idle: the loop has drained every slot)
    (void)hipSetDevice(srv->device);
    for (auto& kv : srv->graphs)
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    for (auto& s : srv->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.ev) (void)hipEventDestroy(s.ev);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.h_buf) (void)hipHostFree(s.h_buf);
        if (s.h_out) (void)hipHostFree(s.h_out);
        if (s.d_buf) (void)dev_release(s.d_buf);
        if (s.d_out) (void)dev_release(s.d_out);
    }
    delete srv;
}

extern "C" {

int tang_server_create(int device, const tang_server_cfg_t* cfg, tang_server_t** out) {
    try {
        if (!out) return fail(TANG_EINVAL, "out is NULL");
        *out = nullptr;
        int count = 0;
        hipError_t ec = hipGetDeviceCount(&count);
        if (ec != hipSuccess) return hip_fail(ec, "hipGetDeviceCount");
        if (count == 0) return fail(TANG_EDEVICE, "no HIP device available");
        if (device < 0 || device >= count) return fail(TANG_EINVAL, "bad device ordinal");
        tang_server_cfg_t c{};
        if (cfg) c = *cfg;
        if (c.n_streams == 0) c.n_streams = 4;
        if (c.max_batch == 0) c.max_batch = 65536;
        if (c.n_streams > 8) return fail(TANG_EINVAL, "n_streams must be 1..8");
        if (c.max_batch < 32 || (c.max_batch & (c.max_batch - 1)))
            return fail(TANG_EINVAL, "max_batch must be a power of two >= 32");
        if (c.max_inflight_packets == 0) c.max_inflight_packets = c.n_streams * c.max_batch;
        if (c.mem_budget_bytes == 0) c.mem_budget_bytes = (size_t)c.n_streams * c.max_batch * kPktBytes;
        auto* srv = new tang_server_t();
        srv->device = device;
        srv->cfg = c;
        srv->slots.resize(c.n_streams);
        hipError_t e = hipSetDevice(device);
        for (auto& s : srv->slots) {
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
            const size_t stage = ((size_t)c.max_batch + 1) * sizeof(tang_header_t);
            if (e == hipSuccess) e = hipHostMalloc((void**)&s.h_buf, stage, hipHostMallocCoherent);
            if (e == hipSuccess)
                e = hipHostMalloc((void**)&s.h_out, c.max_batch * sizeof(uint32_t), hipHostMallocCoherent);
            if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&s.dh_buf, s.h_buf, 0);
            if (e == hipSuccess) e = hipHostGetDevicePointer((void**)&s.dh_out, s.h_out, 0);
            if (e == hipSuccess) e = dev_alloc(&s.d_buf, stage);
            if (e == hipSuccess) e = dev_alloc(&s.d_out, c.max_batch * sizeof(uint32_t));
            if (e == hipSuccess) e = hipMemset(s.d_buf, 0, stage);
        }
        if (e != hipSuccess) {
            free_server(srv);
            return hip_fail(e, "tang_server_create");
        }
        try {
            srv->copies.reset(new CopyPool(kCopyHelpers));
            for (auto& sl : srv->slots) srv->issuers.emplace_back(new SlotIssuer(device, &sl));
            srv->th = std::thread([srv] { srv->loop(); });
        } catch (...) {
            free_server(srv);
            return fail(TANG_ENOMEM, "could not start the serving threads");
        }
        *out = srv;
        return TANG_OK;
    } catch (const std::bad_alloc&) {
        return fail(TANG_ENOMEM, "host allocation failed");
    } catch (...) {
        return fail(TANG_EINVAL, "internal error");
    }
}

int tang_server_add_ruleset(tang_server_t* srv, tang_ruleset_t* rs, uint32_t* tag) {
    if (!srv || !rs || !tag) return fail(TANG_EINVAL, "NULL argument");
    if (rs->device != srv->device) return fail(TANG_EINVAL, "ruleset lives on another device");
    std::lock_guard<std::mutex> g(srv->mu);
    *tag = (uint32_t)srv->rulesets.size();
    srv->rulesets.push_back(rs);
    srv->warmed.push_back(0);
    srv->prepared.push_back(0);
    return TANG_OK;
}

int tang_server_prepare(tang_server_t* srv, uint32_t tag) {
    if (!srv) return fail(TANG_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    if (tag >= srv->rulesets.size()) return fail(TANG_EINVAL, "unknown ruleset tag");
    if (srv->stop) return fail(TANG_EBUSY, "server is stopping");
    if (srv->prepared[tag] == 0) srv->prepared[tag] = 1;
    srv->cv.notify_all();
    srv->prepared_cv.wait(lk, [&] { return srv->prepared[tag] == 2 || srv->stop; });
    if (srv->prepared[tag] != 2) return fail(TANG_EBUSY, "server stopped before the ruleset was prepared");
    return TANG_OK;
}

int tang_server_submit(tang_server_t* srv, uint32_t tag, const tang_header_t* hdr, size_t n,
                       uint32_t* out, tang_req_t** req) {
    try {
        if (!srv || !req) return fail(TANG_EINVAL, "NULL argument");
        *req = nullptr;
        if (n && (!hdr || !out)) return fail(TANG_EINVAL, "NULL buffer");
        auto st = std::make_shared<ReqState>();
        st->tag = tag;
        st->hdr = hdr;
        st->n = n;
        st->out = out;
        st->t_submit = now_ns();
        {
            std::lock_guard<std::mutex> g(srv->mu);
            if (tag >= srv->rulesets.size()) return fail(TANG_EINVAL, "unknown ruleset tag");
            if (n > srv->cfg.max_batch || n > srv->cfg.max_inflight_packets ||
                n * kPktBytes > srv->cfg.mem_budget_bytes)
                return fail(TANG_EBUSY, "request larger than the server's limits");
            if (srv->stop) return fail(TANG_EBUSY, "server is stopping");
            if (n == 0) {
                st->t_admit = st->t_done = st->t_submit;
                st->done = true;
            } else {
                srv->pending.push_back(st);
            }
        }
        srv->cv.notify_all();
        *req = new tang_req_t{st};
        return TANG_OK;
    } catch (const std::bad_alloc&) {
        return fail(TANG_ENOMEM, "host allocation failed");
    }
}

int tang_server_wait(tang_req_t* req, int64_t timeout_us) {
    if (!req) return fail(TANG_EINVAL, "NULL request");
    auto& st = *req->st;
    std::unique_lock<std::mutex> lk(st.mu);
    if (timeout_us < 0) {
        st.cv.wait(lk, [&] { return st.done; });
    } else if (!st.cv.wait_for(lk, std::chrono::microseconds(timeout_us), [&] { return st.done; })) {
        return fail(TANG_ETIMEOUT, "request not done yet");
    }
    if (st.status != TANG_OK) return fail(st.status, "request failed on the device");
    return TANG_OK;
}

int tang_server_poll(const tang_req_t* req) {
    if (!req) return 0;
    std::lock_guard<std::mutex> g(req->st->mu);
    return req->st->done ? 1 : 0;
}

int tang_server_req_times(const tang_req_t* req, uint64_t* submit_ns, uint64_t* admit_ns,
                          uint64_t* done_ns) {
    if (!req) return fail(TANG_EINVAL, "NULL request");
    std::lock_guard<std::mutex> g(req->st->mu);
    if (submit_ns) *submit_ns = req->st->t_submit;
    if (admit_ns) *admit_ns = req->st->t_admit;
    if (done_ns) *done_ns = req->st->t_done;
    return TANG_OK;
}

void tang_server_req_free(tang_req_t* req) { delete req; }

int tang_server_destroy(tang_server_t* srv) {
    if (!srv) return fail(TANG_EINVAL, "NULL server");
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    if (srv->th.joinable()) srv->th.join();
    free_server(srv);
    return TANG_OK;
}

}  // extern "C"
