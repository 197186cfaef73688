// The search stage on the host: the paper's own CPU-GPU split (Sec. 5.1.2, the GPU
// predicts and the CPU searches), kept as a comparison mode for the all-GPU path.
// Per header, following the two-stage classification of Sec. 5.1.1 on the host tuple
// space: probe the predicted tuples (masked key -> bucket -> its rules in (priority, id)
// order, the first match is the bucket's best); then
//   paper mode:  if nothing matched, the ordered search over the remaining tuples
//                (ascending best key, stopping once a tuple's best key cannot beat the
//                answer) -- a lower-priority match in a predicted tuple is returned as is;
//   exact mode:  the same ordered search whether or not a predicted tuple matched, which
//                visits every tuple that could hold a better rule.
// Threads split the headers into contiguous ranges.
#include <algorithm>
#include <thread>
#include <vector>

#include "tang_internal.hpp"

namespace tang {
namespace {

struct HostBest {
    uint64_t key = ~0ull;
    uint32_t id = TANG_NO_MATCH;
    uint32_t tuple = 0;
};

struct HostCounts {
    uint64_t probes = 0, records = 0, top1 = 0, fallbacks = 0, nomatch = 0;
};

inline bool host_match(const tang_rule_t& r, const tang_header_t& p) {
    return ((p.sip ^ r.sip) & pmask(r.sip_len)) == 0 && ((p.dip ^ r.dip) & pmask(r.dip_len)) == 0 &&
           p.sp >= r.sp_lo && p.sp <= r.sp_hi && p.dp >= r.dp_lo && p.dp <= r.dp_hi &&
           (r.proto_mask == 0 || p.proto == r.proto);
}

void scan_members(const tang_ruleset_t* rs, const tang_ruleset_t::Bucket& bk, uint32_t t,
                  const tang_header_t& p, HostBest& b, HostCounts& c) {
    for (uint32_t h : bk.members) {
        const tang_rule_t& r = rs->rules[h].r;
        ++c.records;
        const uint64_t k = key_of(r);
        if (k >= b.key) return;
        if (host_match(r, p)) {
            b.key = k;
            b.id = r.id;
            b.tuple = t;
            return;
        }
    }
}

void probe_host(const tang_ruleset_t* rs, uint32_t t, const tang_header_t& p, HostBest& b,
                HostCounts& c) {
    const auto& sg = rs->sigs[t];
    auto it = rs->bucket_of.find({t, p.sip & pmask(sg.first), p.dip & pmask(sg.second)});
    if (it == rs->bucket_of.end()) return;
    ++c.probes;
    const uint32_t bi = it->second;
    const auto& bk = rs->buckets[bi];
    if (!bk.split) {
        scan_members(rs, bk, t, p, b, c);
        return;
    }
    const uint32_t keys[4][2] = {{kSubDp, p.dp}, {kSubSp, p.sp}, {kSubProto, p.proto}, {kSubRest, 0u}};
    for (const auto& q : keys) {
        auto s = rs->bucket_of.find({t | (q[0] << kKindShift), bi, q[1]});
        if (s != rs->bucket_of.end()) scan_members(rs, rs->buckets[s->second], t, p, b, c);
    }
}

}  // namespace

int search_host(const tang_ruleset_t* rs, const tang_header_t* hdr, const uint32_t* cand,
                uint32_t* out, size_t n, uint32_t kcand, uint32_t threads, bool exact,
                tang_stats_t* stats) {
    const uint32_t ntup = (uint32_t)rs->sigs.size();
    const uint32_t cb = cand_bits((int)ntup);   // as packed by the predictor (see tang_predict)
    std::vector<uint32_t> order(ntup);
    for (uint32_t t = 0; t < ntup; ++t) order[t] = t;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return rs->tuple_best[a] < rs->tuple_best[b]; });
    if (threads == 0) threads = 1;
    threads = (uint32_t)std::min<size_t>(threads, std::max<size_t>(1, n / 1024));
    std::vector<HostCounts> counts(threads);
    auto work = [&](uint32_t w) {
        const size_t lo = n * w / threads, hi = n * (w + 1) / threads;
        HostCounts& c = counts[w];
        for (size_t i = lo; i < hi; ++i) {
            const tang_header_t& p = hdr[i];
            HostBest b;
            uint32_t probed[4], n_probed = 0, c0 = ~0u;
            auto was_probed = [&](uint32_t t) {
                for (uint32_t j = 0; j < n_probed; ++j)
                    if (probed[j] == t) return true;
                return false;
            };
            for (uint32_t k = 0; k < kcand; ++k) {
                const uint32_t t = (cand[i] >> (cb * k)) & ((1u << cb) - 1u);
                if (k == 0) c0 = t;
                if (t >= ntup || was_probed(t)) continue;
                probed[n_probed++] = t;
                probe_host(rs, t, p, b, c);
            }
            const bool found = b.id != TANG_NO_MATCH;
            if (!found) ++c.fallbacks;
            if (exact || !found) {
                for (uint32_t t : order) {
                    if (rs->tuple_best[t] >= b.key) break;
                    if (was_probed(t)) continue;
                    probe_host(rs, t, p, b, c);
                }
            }
            out[i] = b.id;
            if (b.id == TANG_NO_MATCH) ++c.nomatch;
            else if (found && b.tuple == c0) ++c.top1;
        }
    };
    std::vector<std::thread> pool;
    for (uint32_t w = 1; w < threads; ++w) pool.emplace_back(work, w);
    work(0);
    for (auto& th : pool) th.join();
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        stats->packets = n;
        for (const auto& c : counts) {
            stats->probes += c.probes;
            stats->records += c.records;
            stats->top1_hits += c.top1;
            stats->fallbacks += c.fallbacks;
            stats->no_match += c.nomatch;
        }
    }
    return TANG_OK;
}

}  // namespace tang
