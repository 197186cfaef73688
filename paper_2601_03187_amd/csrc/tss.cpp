// Host side of the tuple space: construction (Sec. 4.3), restricted insertion and
// deletion (Sec. 5.2.1), and the device deltas they produce.
#include <algorithm>
#include <numeric>

#include "tang_internal.hpp"

namespace tang {

namespace {

uint32_t next_pow2(uint64_t v) {
    uint64_t p = 1;
    while (p < v) p <<= 1;
    return (uint32_t)p;
}

bool key_less(const tang_rule_t& a, const tang_rule_t& b) { return key_of(a) < key_of(b); }

// Slot contents of bucket b: a split marker, or the bucket's list.
Slot slot_value(const tang_ruleset_t* rs, uint32_t b) {
    const auto& bk = rs->buckets[b];
    if (bk.split) return Slot{bk.ms, bk.md, bk.t << kTlShift, kSplit | b};
    return Slot{bk.ms, bk.md, (bk.t << kTlShift) | (uint32_t)bk.members.size(), bk.off};
}

// Linear probing from the hash position to the first empty slot.
uint32_t slot_insert(std::vector<Slot>& slots, const Slot& v) {
    uint32_t mask = (uint32_t)slots.size() - 1;
    uint32_t h = slot_of(key_hash(v.tl >> kTlShift, v.ms, v.md)) & mask;
    while (slots[h].tl != kEmptyTL) h = (h + 1) & mask;
    slots[h] = v;
    return h;
}

bool is_main(const tang_ruleset_t::Bucket& bk) { return (bk.t >> kKindShift) == 0; }

// Sub-list key of rule r inside the split main bucket b of tuple t.
tang_ruleset_t::BKey sub_key_of(uint32_t t, uint32_t b, const tang_rule_t& r) {
    if (r.dp_lo == r.dp_hi) return {t | (kSubDp << kKindShift), b, r.dp_lo};
    if (r.sp_lo == r.sp_hi) return {t | (kSubSp << kKindShift), b, r.sp_lo};
    if (r.proto_mask) return {t | (kSubProto << kKindShift), b, r.proto};
    return {t | (kSubRest << kKindShift), b, 0u};
}
tang_ruleset_t::BKey sub_key(const tang_ruleset_t* rs, uint32_t b, uint32_t h) {
    return sub_key_of(rs->buckets[b].t, b, rs->rules[h].r);
}

uint32_t find_or_add_bucket(tang_ruleset_t* rs, const tang_ruleset_t::BKey& k) {
    auto it = rs->bucket_of.find(k);
    if (it != rs->bucket_of.end()) return it->second;
    const uint32_t b = (uint32_t)rs->buckets.size();
    rs->buckets.push_back({k.t, k.ms, k.md, 0, 0, 0, {}, false});
    rs->bucket_of.emplace(k, b);
    return b;
}

// Moves the rules of main bucket b into its sub-lists (order kept); returns every
// bucket whose contents changed (b itself and the sub-lists).
std::vector<uint32_t> split_bucket(tang_ruleset_t* rs, uint32_t b) {
    std::vector<uint32_t> touched{b};
    std::vector<uint32_t> mem;
    mem.swap(rs->buckets[b].members);
    rs->buckets[b].split = true;
    for (uint32_t h : mem) {
        const uint32_t sb = find_or_add_bucket(rs, sub_key(rs, b, h));
        auto& sm = rs->buckets[sb].members;
        auto pos = std::upper_bound(sm.begin(), sm.end(), h, [&](uint32_t a, uint32_t x) {
            return key_of(rs->rules[a].r) < key_of(rs->rules[x].r);
        });
        sm.insert(pos, h);
        rs->rules[h].bucket = sb;
        if (std::find(touched.begin(), touched.end(), sb) == touched.end()) touched.push_back(sb);
    }
    return touched;
}

// The filter bit of a main bucket: in the block its group value picks (tuple (0, 0)
// has no group: its one possible key always has a bucket).
void filter_add(tang_ruleset_t* rs, const tang_ruleset_t::Bucket& bk) {
    const uint32_t ls = rs->sigs[bk.t].first, ld = rs->sigs[bk.t].second;
    if (ls == 0 && ld == 0) return;
    const uint32_t gk = group_key_of(ls, ld);
    const uint32_t v = gk & 64u ? bk.md : bk.ms, o = gk & 64u ? bk.ms : bk.md;
    const uint32_t blocks = (uint32_t)rs->filter.size() / 2;
    const uint32_t blk = filter_block(gk, v) & (blocks - 1u), bits = filter_bits(bk.t, o);
    for (uint32_t bit : {bits & 63u, bits >> 8}) rs->filter[2 * blk + (bit >> 5)] |= 1u << (bit & 31u);
}

// Slot table at load <= 1/4 (short walks) and the bucket filter at >= 32 bits per bucket
// (blocks of 64 bits).
void rebuild_slots(tang_ruleset_t* rs) {
    const uint64_t nb = rs->buckets.size();
    rs->slots.assign(next_pow2(std::max<uint64_t>(1024, 4 * nb + 4)), Slot{0, 0, kEmptyTL, 0});
    rs->filter.assign(2 * (uint64_t)next_pow2(std::max<uint64_t>(1024, (nb + 1) / 2)), 0u);
    for (uint32_t b = 0; b < rs->buckets.size(); ++b) {
        auto& bk = rs->buckets[b];
        bk.slot = slot_insert(rs->slots, slot_value(rs, b));
        if (is_main(bk)) filter_add(rs, bk);
    }
}

// Restricted insertion (Sec. 5.2.1): identical signature, else the first tuple with the
// largest length sum among those with every length <= the rule's; -1 if none.
int choose_tuple(const std::vector<std::pair<uint8_t, uint8_t>>& sigs, uint8_t sl, uint8_t dl) {
    for (size_t i = 0; i < sigs.size(); ++i)
        if (sigs[i].first == sl && sigs[i].second == dl) return (int)i;
    int best = -1, best_sum = -1;
    for (size_t i = 0; i < sigs.size(); ++i) {
        if (sigs[i].first <= sl && sigs[i].second <= dl) {
            int s = sigs[i].first + sigs[i].second;
            if (s > best_sum) { best = (int)i; best_sum = s; }
        }
    }
    return best;
}

}  // namespace

int validate_rule(const tang_rule_t& r) {
    if (r.sip_len > 32 || r.dip_len > 32) return fail(TANG_EINVAL, "prefix length > 32");
    if (r.sp_lo > r.sp_hi || r.dp_lo > r.dp_hi) return fail(TANG_EINVAL, "port range lo > hi");
    if (r.proto_mask != 0 && r.proto_mask != 0xFF)
        return fail(TANG_EINVAL, "proto_mask must be 0 or 0xFF");
    if (r.id == TANG_NO_MATCH) return fail(TANG_EINVAL, "rule id 0xFFFFFFFF is reserved");
    return TANG_OK;
}

tang_rule_t normalise(const tang_rule_t& r) {
    tang_rule_t n = r;
    n.sip &= pmask(r.sip_len);
    n.dip &= pmask(r.dip_len);
    if (n.proto_mask == 0) n.proto = 0;
    return n;
}

Rec make_rec(const tang_ruleset_t* rs, uint32_t h) {
    const auto& hr = rs->rules[h];
    const tang_rule_t& r = hr.r;
    Rec x;
    x.sip = r.sip;
    x.dip = r.dip;
    x.sp = (uint32_t)r.sp_lo | ((uint32_t)r.sp_hi << 16);
    x.dp = (uint32_t)r.dp_lo | ((uint32_t)r.dp_hi << 16);
    // a rule held by a coarser tuple than its own signature (restricted insertion) has
    // its prefixes checked in the scan; in its own tuple the bucket key implies them
    const auto& sig = rs->sigs[hr.tuple];
    const uint32_t check = (sig.first != r.sip_len || sig.second != r.dip_len) ? 1u : 0u;
    x.meta = meta_pack(r.sip_len, r.dip_len, r.proto, r.proto_mask ? 1u : 0u, hr.tuple, check);
    x.cmask = 0;
    x.prio = r.priority;
    x.id = r.id;
    return x;
}

static Rec dead_rec() {
    Rec x;
    std::memset(&x, 0, sizeof x);
    x.prio = kDead;
    x.id = kDead;
    return x;
}

TupleTable make_tuple_table(const tang_ruleset_t* rs) {
    TupleTable tt;
    std::memset(&tt, 0, sizeof tt);
    uint32_t n = (uint32_t)rs->sigs.size();
    for (uint32_t t = 0; t < n; ++t) {
        tt.t[t].smask = pmask(rs->sigs[t].first);
        tt.t[t].dmask = pmask(rs->sigs[t].second);
        tt.t[t].best_prio = (uint32_t)(rs->tuple_best[t] >> 32);
        tt.t[t].best_id = (uint32_t)rs->tuple_best[t];
    }
    std::vector<uint32_t> ord(n);
    std::iota(ord.begin(), ord.end(), 0u);
    std::stable_sort(ord.begin(), ord.end(),
                     [&](uint32_t a, uint32_t b) { return rs->tuple_best[a] < rs->tuple_best[b]; });
    for (uint32_t i = 0; i < n; ++i) {
        tt.order[i] = (uint16_t)ord[i];
        tt.rank_prio[i] = (uint32_t)(rs->tuple_best[ord[i]] >> 32);
        tt.rank_id[i] = (uint32_t)rs->tuple_best[ord[i]];
        for (int w = 0; w < kMaxWords; ++w) tt.prefix[i + 1][w] = tt.prefix[i][w];
        tt.prefix[i + 1][ord[i] >> 5] |= 1u << (ord[i] & 31u);
    }
    tt.n = n;
    for (uint32_t t = 0; t < n; ++t) tt.all_mask[t >> 5] |= 1u << (t & 31u);
    tt.nw = rs->nw;
    // filter groups in order of first appearance over the tuples
    for (uint32_t t = 0; t < n; ++t) {
        const uint32_t ls = rs->sigs[t].first, ld = rs->sigs[t].second;
        if (ls == 0 && ld == 0) {
            tt.gid[t] = (uint8_t)kNoGroup;
            tt.nogroup[t >> 5] |= 1u << (t & 31u);
            continue;
        }
        const uint32_t gk = group_key_of(ls, ld);
        uint32_t g = 0;
        while (g < tt.ngroups && tt.gkey[g] != gk) ++g;
        if (g == tt.ngroups) tt.gkey[tt.ngroups++] = gk;
        tt.gid[t] = (uint8_t)g;
        tt.gmask[g][t >> 5] |= 1u << (t & 31u);
    }
    tt.slot_mask = rs->slots.empty() ? 0 : (uint32_t)rs->slots.size() - 1;
    tt.filter_mask = rs->filter.empty() ? 0 : (uint32_t)rs->filter.size() / 2u - 1u;
    return tt;
}

int build_host(tang_ruleset_t* rs, const tang_rule_t* rules, size_t n) {
    if (n && !rules) return fail(TANG_EINVAL, "rules is NULL");
    if (n > 0x7FFFFFFFu) return fail(TANG_EINVAL, "too many rules");
    rs->rules.reserve(n);
    rs->id2h.reserve(n * 2 + 16);
    for (size_t i = 0; i < n; ++i) {
        int rc = validate_rule(rules[i]);
        if (rc) return rc;
        if (!rs->id2h.emplace(rules[i].id, (uint32_t)i).second)
            return fail(TANG_EEXIST, "repeated rule id " + std::to_string(rules[i].id));
        rs->rules.push_back({normalise(rules[i]), 0, 0, 0, true});
    }
    rs->n_live = n;

    std::vector<uint32_t> order(n);
    std::iota(order.begin(), order.end(), 0u);
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return key_less(rs->rules[a].r, rs->rules[b].r);
    });

    // Tuples by first appearance in (priority, id) order (Table 1 numbering).
    for (uint32_t h : order) {
        auto& hr = rs->rules[h];
        std::pair<uint8_t, uint8_t> sig(hr.r.sip_len, hr.r.dip_len);
        size_t t = 0;
        while (t < rs->sigs.size() && rs->sigs[t] != sig) ++t;
        if (t == rs->sigs.size()) {
            if (rs->sigs.size() == TANG_MAX_TUPLES)
                return fail(TANG_EINVAL, "more than " + std::to_string(TANG_MAX_TUPLES) +
                                             " distinct (sip_len, dip_len) signatures");
            rs->sigs.push_back(sig);
            rs->tuple_best.push_back(key_of(hr.r));
        }
        hr.tuple = (uint32_t)t;
    }
    rs->nw = words_for(rs->sigs.size());

    // Buckets keyed by (tuple, masked SIP, masked DIP), members in key order.
    for (uint32_t h : order) {
        auto& hr = rs->rules[h];
        uint32_t t = hr.tuple;
        tang_ruleset_s::BKey k{t, hr.r.sip & pmask(rs->sigs[t].first), hr.r.dip & pmask(rs->sigs[t].second)};
        const uint32_t b = find_or_add_bucket(rs, k);
        rs->buckets[b].members.push_back(h);
        hr.bucket = b;
    }
    const size_t n_main = rs->buckets.size();
    for (uint32_t b = 0; b < n_main; ++b)
        if (rs->buckets[b].members.size() > kSplitAt) split_bucket(rs, b);
    // Records: buckets laid out contiguously in creation order (by their best key).
    uint32_t off = 0;
    for (auto& bk : rs->buckets) {
        if (bk.members.size() > kMaxBucketLen) return fail(TANG_ENOMEM, "bucket too long");
        bk.off = off;
        bk.cap = (uint32_t)bk.members.size();
        for (uint32_t i = 0; i < bk.cap; ++i) rs->rules[bk.members[i]].pos = off + i;
        off += bk.cap;
    }
    rs->rec_used = off;
    rs->rec_cap = off + std::max<uint32_t>(65536u, off / 4);
    rebuild_slots(rs);
    return TANG_OK;
}

// ---------------------------------------------------------------------------------------
// Device upload of a freshly built ruleset, with the conflict masks computed on the GPU.

int upload_all(tang_ruleset_t* rs) {
    TANG_HIP(hipSetDevice(rs->device));
    hipStream_t s = rs->upd_stream;
    TANG_HIP(dev_alloc(&rs->d_slots, rs->slots.size() * sizeof(Slot)));
    TANG_HIP(dev_alloc(&rs->d_filter, rs->filter.size() * sizeof(uint32_t)));
    TANG_HIP(hipMemcpy(rs->d_filter, rs->filter.data(), rs->filter.size() * sizeof(uint32_t),
                       hipMemcpyHostToDevice));
    TANG_HIP(dev_alloc(&rs->d_recs, (size_t)rs->rec_cap * sizeof(Rec)));
    if (rs->nw > 1) {
        TANG_HIP(dev_alloc(&rs->d_cmask, (size_t)rs->rec_cap * rs->nw * sizeof(uint32_t)));
        TANG_HIP(hipMemset(rs->d_cmask, 0, (size_t)rs->rec_cap * rs->nw * sizeof(uint32_t)));
    }
    TANG_HIP(dev_alloc(&rs->d_tt, sizeof(TupleTable)));
    TANG_HIP(dev_alloc(&rs->d_stats, kStatCopies * sizeof(StatsDev)));

    std::vector<Rec> recs(rs->rec_cap, dead_rec());
    for (uint32_t h = 0; h < rs->rules.size(); ++h)
        if (rs->rules[h].live) recs[rs->rules[h].pos] = make_rec(rs, h);
    TupleTable tt = make_tuple_table(rs);
    TANG_HIP(hipMemcpy(rs->d_slots, rs->slots.data(), rs->slots.size() * sizeof(Slot),
                       hipMemcpyHostToDevice));
    TANG_HIP(hipMemcpy(rs->d_recs, recs.data(), recs.size() * sizeof(Rec), hipMemcpyHostToDevice));
    TANG_HIP(hipMemcpy(rs->d_tt, &tt, sizeof tt, hipMemcpyHostToDevice));

    // Boxes of the live rules in ascending key order for the pairwise mask kernel.
    std::vector<uint32_t> order;
    order.reserve(rs->n_live);
    for (uint32_t h = 0; h < rs->rules.size(); ++h)
        if (rs->rules[h].live) order.push_back(h);
    std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return key_of(rs->rules[a].r) < key_of(rs->rules[b].r);
    });
    if (!order.empty()) {
        std::vector<BoxDev> boxes(order.size());
        for (size_t i = 0; i < order.size(); ++i) {
            const auto& hr = rs->rules[order[i]];
            const tang_rule_t& r = hr.r;
            uint32_t sm = pmask(r.sip_len), dm = pmask(r.dip_len);
            boxes[i] = BoxDev{r.sip, r.sip | ~sm, r.dip, r.dip | ~dm,
                              (uint32_t)r.sp_lo | ((uint32_t)r.sp_hi << 16),
                              (uint32_t)r.dp_lo | ((uint32_t)r.dp_hi << 16),
                              (uint32_t)r.proto | ((r.proto_mask ? 1u : 0u) << 8) | (hr.tuple << 16),
                              hr.pos};
        }
        BoxDev* d_boxes = nullptr;
        TANG_HIP(dev_alloc(&d_boxes, boxes.size() * sizeof(BoxDev)));
        hipError_t e = hipMemcpy(d_boxes, boxes.data(), boxes.size() * sizeof(BoxDev),
                                 hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = launch_conflict_build(d_boxes, boxes.size(), rs->d_recs, rs->d_cmask, rs->nw,
                                      rs->d_tt->all_mask, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        (void)dev_release(d_boxes);
        if (e != hipSuccess) return hip_fail(e, "conflict-mask build");
    }
    return TANG_OK;
}

// ---------------------------------------------------------------------------------------
// Updates.

namespace {

// Rewrites the given buckets on the device: each keeps its slot, its records are
// re-laid in member order (in place if they fit, else at the end of the record array),
// freed record positions are marked dead, conflict masks of moved rules move with them.
// `fresh` are handles of rules not yet on the device. Then the slot entries, tuple
// table, and the conflict masks of the fresh rules are brought up to date.
int flush(tang_ruleset_t* rs, const std::vector<uint32_t>& dirty, const std::vector<uint32_t>& fresh,
          bool rehash, bool filter_dirty) {
    rs->version++;
    if (rs->device == TANG_HOST_ONLY) return TANG_OK;
    TANG_HIP(hipSetDevice(rs->device));
    hipStream_t s = rs->upd_stream;
    std::vector<char> is_fresh(rs->rules.size(), 0);
    for (uint32_t h : fresh) is_fresh[h] = 1;

    std::vector<uint32_t> src, dst;   // src: old position, or kNew | index into newrecs
    std::vector<Rec> newrecs;
    const uint32_t kNew = 0x80000000u;
    std::vector<uint32_t> touched_slots;
    uint32_t need_end = rs->rec_used;
    // first pass: capacity planning
    for (uint32_t b : dirty) {
        auto& bk = rs->buckets[b];
        uint32_t len = (uint32_t)bk.members.size();
        if (len > bk.cap) need_end += len + std::max<uint32_t>(4u, len / 2);
    }
    if (need_end > rs->rec_cap) {
        uint32_t ncap = std::max<uint32_t>(need_end + need_end / 2, rs->rec_cap * 2);
        Rec* nrec = nullptr;
        TANG_HIP(dev_alloc(&nrec, (size_t)ncap * sizeof(Rec)));
        TANG_HIP(hipMemcpyAsync(nrec, rs->d_recs, (size_t)rs->rec_used * sizeof(Rec),
                                hipMemcpyDeviceToDevice, s));
        std::vector<Rec> tail(ncap - rs->rec_used, dead_rec());
        TANG_HIP(hipMemcpyAsync(nrec + rs->rec_used, tail.data(), tail.size() * sizeof(Rec),
                                hipMemcpyHostToDevice, s));
        if (rs->nw > 1) {
            uint32_t* nmask = nullptr;
            const size_t row = rs->nw * sizeof(uint32_t);
            TANG_HIP(dev_alloc(&nmask, (size_t)ncap * row));
            TANG_HIP(hipMemsetAsync(nmask, 0, (size_t)ncap * row, s));
            TANG_HIP(hipMemcpyAsync(nmask, rs->d_cmask, (size_t)rs->rec_used * row,
                                    hipMemcpyDeviceToDevice, s));
            TANG_HIP(hipStreamSynchronize(s));
            TANG_HIP(dev_release(rs->d_cmask));
            rs->d_cmask = nmask;
        }
        TANG_HIP(hipStreamSynchronize(s));
        TANG_HIP(dev_release(rs->d_recs));
        rs->d_recs = nrec;
        rs->rec_cap = ncap;
    }
    for (uint32_t b : dirty) {
        auto& bk = rs->buckets[b];
        uint32_t len = (uint32_t)bk.members.size();
        uint32_t old_off = bk.off, old_cap = bk.cap;
        if (len > bk.cap) {
            bk.off = rs->rec_used;
            bk.cap = len + std::max<uint32_t>(4u, len / 2);
            rs->rec_used += bk.cap;
            for (uint32_t i = len; i < bk.cap; ++i) {  // new slack: dead
                src.push_back(kNew | (uint32_t)newrecs.size());
                dst.push_back(bk.off + i);
                newrecs.push_back(dead_rec());
            }
        }
        for (uint32_t i = 0; i < len; ++i) {
            uint32_t h = bk.members[i];
            auto& hr = rs->rules[h];
            if (is_fresh[h]) {
                src.push_back(kNew | (uint32_t)newrecs.size());
                newrecs.push_back(make_rec(rs, h));
            } else {
                src.push_back(hr.pos);
            }
            dst.push_back(bk.off + i);
            hr.pos = bk.off + i;
        }
        // vacated positions of the old region
        uint32_t keep_lo = (bk.off == old_off) ? len : 0;
        for (uint32_t i = keep_lo; i < old_cap; ++i) {
            src.push_back(kNew | (uint32_t)newrecs.size());
            dst.push_back(old_off + i);
            newrecs.push_back(dead_rec());
        }
        rs->slots[bk.slot] = slot_value(rs, b);
        touched_slots.push_back(bk.slot);
    }

    std::vector<void*> tmp;
    std::vector<Slot> vals;   // host sources of async copies: alive until the final sync
    std::vector<uint32_t> pos;
    auto dev_copy = [&](const void* host, size_t bytes, void** out) -> hipError_t {
        *out = nullptr;
        if (!bytes) return hipSuccess;
        hipError_t e = dev_alloc(out, bytes);
        if (e != hipSuccess) return e;
        tmp.push_back(*out);
        return hipMemcpyAsync(*out, host, bytes, hipMemcpyHostToDevice, s);
    };
    hipError_t e = hipSuccess;
    void *d_src = nullptr, *d_dst = nullptr, *d_new = nullptr, *d_stage = nullptr;
    if (!dst.empty()) {
        e = dev_copy(src.data(), src.size() * 4, &d_src);
        if (e == hipSuccess) e = dev_copy(dst.data(), dst.size() * 4, &d_dst);
        if (e == hipSuccess && !newrecs.empty())
            e = dev_copy(newrecs.data(), newrecs.size() * sizeof(Rec), &d_new);
        if (e == hipSuccess) {
            e = dev_alloc(&d_stage, dst.size() * sizeof(Rec));
            if (e == hipSuccess) tmp.push_back(d_stage);
        }
        if (e == hipSuccess)
            e = launch_move_records(rs->d_recs, (const Rec*)d_new, (const uint32_t*)d_src,
                                    (const uint32_t*)d_dst, (uint32_t)dst.size(), (Rec*)d_stage, s);
        if (e == hipSuccess && rs->nw > 1) {
            void* d_mstage = nullptr;
            e = dev_alloc(&d_mstage, dst.size() * rs->nw * sizeof(uint32_t));
            if (e == hipSuccess) {
                tmp.push_back(d_mstage);
                e = launch_move_masks(rs->d_cmask, rs->nw, (const uint32_t*)d_src, (const uint32_t*)d_dst,
                                      (uint32_t)dst.size(), (uint32_t*)d_mstage, s);
            }
        }
    }
    // slots
    if (e == hipSuccess) {
        if (rehash) {
            Slot* ns = nullptr;
            uint32_t* nf = nullptr;
            e = hipStreamSynchronize(s);
            if (e == hipSuccess) e = dev_alloc(&ns, rs->slots.size() * sizeof(Slot));
            if (e == hipSuccess) e = dev_alloc(&nf, rs->filter.size() * sizeof(uint32_t));
            if (e == hipSuccess)
                e = hipMemcpyAsync(ns, rs->slots.data(), rs->slots.size() * sizeof(Slot),
                                   hipMemcpyHostToDevice, s);
            if (e == hipSuccess)
                e = hipMemcpyAsync(nf, rs->filter.data(), rs->filter.size() * sizeof(uint32_t),
                                   hipMemcpyHostToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e == hipSuccess) {
                (void)dev_release(rs->d_slots);
                (void)dev_release(rs->d_filter);
                rs->d_slots = ns;
                rs->d_filter = nf;
            } else {
                if (ns) (void)dev_release(ns);
                if (nf) (void)dev_release(nf);
            }
        } else if (!touched_slots.empty()) {
            std::sort(touched_slots.begin(), touched_slots.end());
            touched_slots.erase(std::unique(touched_slots.begin(), touched_slots.end()),
                                touched_slots.end());
            vals.resize(touched_slots.size());
            for (size_t i = 0; i < vals.size(); ++i) vals[i] = rs->slots[touched_slots[i]];
            void *d_idx = nullptr, *d_val = nullptr;
            e = dev_copy(touched_slots.data(), touched_slots.size() * 4, &d_idx);
            if (e == hipSuccess) e = dev_copy(vals.data(), vals.size() * sizeof(Slot), &d_val);
            if (e == hipSuccess)
                e = launch_scatter_slots(rs->d_slots, (const uint32_t*)d_idx, (const Slot*)d_val,
                                         (uint32_t)vals.size(), s);
            if (e == hipSuccess && filter_dirty)
                e = hipMemcpyAsync(rs->d_filter, rs->filter.data(),
                                   rs->filter.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s);
        }
    }
    TupleTable tt = make_tuple_table(rs);
    if (e == hipSuccess) e = hipMemcpyAsync(rs->d_tt, &tt, sizeof tt, hipMemcpyHostToDevice, s);
    // conflict masks of fresh rules, and their bit in lower-priority rules they meet
    if (e == hipSuccess && !fresh.empty()) {
        pos.resize(fresh.size());
        for (size_t i = 0; i < fresh.size(); ++i) pos[i] = rs->rules[fresh[i]].pos;
        void* d_pos = nullptr;
        e = dev_copy(pos.data(), pos.size() * 4, &d_pos);
        if (e == hipSuccess)
            e = launch_conflict_update(rs->d_recs, rs->d_cmask, rs->nw, rs->rec_used,
                                       (const uint32_t*)d_pos, (uint32_t)pos.size(), s);
    }
    hipError_t e2 = hipStreamSynchronize(s);
    for (void* p : tmp) (void)dev_release(p);
    if (e != hipSuccess) return hip_fail(e, "update flush");
    if (e2 != hipSuccess) return hip_fail(e2, "update flush sync");
    return TANG_OK;
}

// The host mirror already holds a batch when its device flush runs; if the flush fails
// (an allocation or a HIP call), host and device disagree, so the ruleset refuses every
// later call that reads its device state (tang_ruleset_export still gives the live rules
// a rebuild starts from).
int flush_or_fail(tang_ruleset_t* rs, const std::vector<uint32_t>& dirty,
                  const std::vector<uint32_t>& fresh, bool rehash, bool filter_dirty) {
    const int rc = flush(rs, dirty, fresh, rehash, filter_dirty);
    if (rc) {
        rs->failed = true;
        return fail(rc, std::string("update not applied on the device (") + tang_last_error() +
                            "); the ruleset is unusable, rebuild it from tang_ruleset_export");
    }
    return TANG_OK;
}

}  // namespace

int apply_insert(tang_ruleset_t* rs, const tang_rule_t* rules, size_t n) {
    if (n == 0) return TANG_OK;
    if (!rules) return fail(TANG_EINVAL, "rules is NULL");
    // Validate the whole batch first (all-or-nothing).
    std::unordered_map<uint32_t, int> seen;
    auto sigs = rs->sigs;
    // Every list must stay within what a slot can describe (kMaxBucketLen): each rule's
    // destination list is bounded by its current length plus the batch's rules bound for
    // it (a main bucket that splits during the batch only sheds rules into sub-lists).
    std::unordered_map<tang_ruleset_s::BKey, size_t, tang_ruleset_s::BKeyHash> list_len;
    for (size_t i = 0; i < n; ++i) {
        int rc = validate_rule(rules[i]);
        if (rc) return rc;
        if (rs->id2h.count(rules[i].id) || !seen.emplace(rules[i].id, 1).second)
            return fail(TANG_EEXIST, "rule id " + std::to_string(rules[i].id) + " is live or repeated");
        int t = choose_tuple(sigs, rules[i].sip_len, rules[i].dip_len);
        if (t < 0) {
            if (sigs.size() == tuple_limit(rs->nw))
                return fail(TANG_EINVAL, "insert would need tuple " + std::to_string(sigs.size() + 1) +
                                             " (the ruleset was built with " + std::to_string(rs->nw) +
                                             " conflict-mask words per rule)");
            t = (int)sigs.size();
            sigs.emplace_back(rules[i].sip_len, rules[i].dip_len);
        }
        const tang_rule_t r = normalise(rules[i]);
        tang_ruleset_s::BKey key{(uint32_t)t, r.sip & pmask(sigs[t].first), r.dip & pmask(sigs[t].second)};
        auto mb = rs->bucket_of.find(key);
        if (mb != rs->bucket_of.end() && rs->buckets[mb->second].split)
            key = sub_key_of((uint32_t)t, mb->second, r);
        auto ins = list_len.emplace(key, 0);
        if (ins.second) {
            auto lb = rs->bucket_of.find(key);
            if (lb != rs->bucket_of.end()) ins.first->second = rs->buckets[lb->second].members.size();
        }
        if (++ins.first->second > kMaxBucketLen)
            return fail(TANG_ENOMEM, "insert would make a bucket list longer than " +
                                         std::to_string(kMaxBucketLen) + " rules");
    }
    std::vector<uint32_t> dirty, fresh;
    std::vector<char> mark(rs->buckets.size() + n, 0);
    size_t nb_before = rs->buckets.size();
    for (size_t i = 0; i < n; ++i) {
        tang_rule_t r = normalise(rules[i]);
        int t = choose_tuple(rs->sigs, r.sip_len, r.dip_len);
        if (t < 0) {
            t = (int)rs->sigs.size();
            rs->sigs.emplace_back(r.sip_len, r.dip_len);
            rs->tuple_best.push_back(key_of(r));
        }
        uint32_t h = (uint32_t)rs->rules.size();
        rs->rules.push_back({r, (uint32_t)t, 0, 0, true});
        rs->id2h[r.id] = h;
        rs->n_live++;
        if (rs->sigs[t] != std::make_pair(r.sip_len, r.dip_len)) rs->n_coarse++;
        rs->tuple_best[t] = std::min(rs->tuple_best[t], key_of(r));
        tang_ruleset_s::BKey k{(uint32_t)t, r.sip & pmask(rs->sigs[t].first),
                               r.dip & pmask(rs->sigs[t].second)};
        const uint32_t mb = find_or_add_bucket(rs, k);
        const uint32_t b = rs->buckets[mb].split ? find_or_add_bucket(rs, sub_key(rs, mb, h)) : mb;
        if (rs->buckets.size() > mark.size()) mark.resize(rs->buckets.size() + n, 0);
        auto& mem = rs->buckets[b].members;
        auto pos = std::upper_bound(mem.begin(), mem.end(), h, [&](uint32_t a, uint32_t x) {
            return key_of(rs->rules[a].r) < key_of(rs->rules[x].r);
        });
        mem.insert(pos, h);
        rs->rules[h].bucket = b;
        std::vector<uint32_t> changed{b};
        if (b == mb && mem.size() > kSplitAt) changed = split_bucket(rs, mb);
        if (rs->buckets.size() > mark.size()) mark.resize(rs->buckets.size() + n, 0);
        for (uint32_t c : changed)
            if (!mark[c]) { mark[c] = 1; dirty.push_back(c); }
        fresh.push_back(h);
    }
    // new buckets need slots; grow the table when it would pass half full
    bool rehash = false, filter_dirty = false;
    if (rs->buckets.size() != nb_before) {
        // keep the slot table at most 1/3 full and the filter at >= half its bits per bucket
        if (3 * rs->buckets.size() + 3 > rs->slots.size() ||
            16 * rs->buckets.size() > rs->filter.size() * 32) {
            rebuild_slots(rs);
            rehash = true;
        } else {
            for (size_t b = nb_before; b < rs->buckets.size(); ++b) {
                auto& bk = rs->buckets[b];
                bk.slot = slot_insert(rs->slots, Slot{bk.ms, bk.md, bk.t << kTlShift, 0});
                if (is_main(bk)) filter_add(rs, bk);
            }
            filter_dirty = true;
        }
    }
    return flush_or_fail(rs, dirty, fresh, rehash, filter_dirty);
}

int apply_delete(tang_ruleset_t* rs, const uint32_t* ids, size_t n) {
    if (n == 0) return TANG_OK;
    if (!ids) return fail(TANG_EINVAL, "ids is NULL");
    std::unordered_map<uint32_t, int> seen;
    for (size_t i = 0; i < n; ++i) {
        if (!rs->id2h.count(ids[i]) || !seen.emplace(ids[i], 1).second)
            return fail(TANG_ENOTFOUND, "rule id " + std::to_string(ids[i]) + " is not live");
    }
    std::vector<uint32_t> dirty;
    std::vector<char> mark(rs->buckets.size(), 0);
    for (size_t i = 0; i < n; ++i) {
        uint32_t h = rs->id2h[ids[i]];
        auto& hr = rs->rules[h];
        auto& mem = rs->buckets[hr.bucket].members;
        mem.erase(std::find(mem.begin(), mem.end(), h));
        hr.live = false;
        rs->id2h.erase(ids[i]);
        rs->n_live--;
        if (rs->sigs[hr.tuple] != std::make_pair(hr.r.sip_len, hr.r.dip_len)) rs->n_coarse--;
        if (!mark[hr.bucket]) { mark[hr.bucket] = 1; dirty.push_back(hr.bucket); }
    }
    return flush_or_fail(rs, dirty, {}, false, false);
}

}  // namespace tang
