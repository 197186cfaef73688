"""Immediate updates on the device (Sec. 5.2.1): after every insert/delete batch the
GPU answers equal the oracle's re-scan of the live rules, bit for bit."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2601_03187_amd import synth, train
from paper_2601_03187_amd import tang as T
from tests._gpu import classify_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _live_mask(all_rules, live_ids):
    return np.isin(all_rules["id"], np.fromiter(live_ids, dtype=np.uint32))


def test_update_rounds_match_oracle():
    """Scaled-down update stream: 20k rules, 8 rounds of 100 inserts + 100 deletes, each
    followed by a 50k-header lookup batch drawn from the live rules; fixed BF16 weights.
    Some inserts use prefix lengths no tuple has (/20, /28), so they land in a coarser
    tuple and their own prefixes are checked in the bucket scan."""
    torch_cuda()
    rules = synth.make_rules(20_000, seed=404)
    rs = T.tang_ruleset_create(0, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        hdr0 = synth.make_packets(rules, 50_000, seed=1, frac_in=0.8)
        Ws, bs, sc, acc = train.fit(rs, rules, hdr0, 256, steps=300, seed=2, device="cuda")
        T.tang_model_load(rs, Ws, bs, "bf16")
        all_rules = rules.copy()
        live = set(int(i) for i in rules["id"])
        ups = synth.make_update_stream(rules, rounds=8, per_round=100, seed=405,
                                       prio_range=len(rules))
        rng = np.random.default_rng(7)
        for rd, (ins, dels) in enumerate(ups):
            odd = rng.random(len(ins)) < 0.3
            ins["sip_len"][odd] = rng.choice([20, 28], odd.sum())
            ins["sip"][odd] &= np.uint32(0xFFFFFFF0)
            T.tang_insert(rs, ins)
            T.tang_delete(rs, dels)
            all_rules = np.concatenate([all_rules, ins])
            live |= set(int(i) for i in ins["id"])
            live -= set(int(i) for i in dels)
            lm = _live_mask(all_rules, live)
            assert T.tang_ruleset_num_rules(rs) == len(live)
            assert T.tang_ruleset_num_tuples(rs) == C  # tuple set unchanged (Sec. 5.2.1)
            pk = synth.make_packets(all_rules[lm], 50_000, seed=100 + rd, frac_in=0.8)
            want = orc.classify(all_rules, pk, live=lm)
            got = classify_dev(rs, pk)
            assert np.array_equal(got, want), rd
        # conflict masks stay sound: a superset of the brute-force masks of the live rules
        small = all_rules[lm]
        pick = rng.choice(len(small), 60, replace=False)
        tup = np.array([T.tang_ruleset_rule_tuple(rs, int(i)) for i in small["id"]])
        for k in pick:
            m = T.tang_ruleset_conflict_mask(rs, int(small[k]["id"]))
            key = (int(small[k]["priority"]), int(small[k]["id"]))
            need = 0
            for j in range(len(small)):
                if (int(small[j]["priority"]), int(small[j]["id"])) < key and orc.boxes_intersect(small[j], small[k]):
                    need |= 1 << int(tup[j])
            assert m & need == need, (k, hex(m), hex(need))
    finally:
        T.tang_ruleset_destroy(rs)


def test_growth_rehash_and_appended_tuple():
    """Many inserts into one bucket (record array grows, the bucket relocates), many new
    buckets (the slot table is rebuilt), and a signature no tuple dominates (a tuple is
    appended; only certification and the fallback can find its rules)."""
    torch_cuda()
    base = synth.make_rules(500, seed=9)
    base["sip_len"] = 32
    base["dip_len"] = 32
    rs = T.tang_ruleset_create(0, base)
    try:
        assert T.tang_ruleset_num_tuples(rs) == 1
        Ws, bs = train.random_weights(1, 128, seed=1)
        T.tang_model_load(rs, Ws, bs, "fp32")
        all_rules = base.copy()
        next_id = 10_000
        rng = np.random.default_rng(3)
        for b in range(6):  # 6 x 12,000 rules into the single (32, 32) tuple
            ins = synth.make_rules(12_000, seed=50 + b, ordering="literal")
            ins["sip_len"] = 32
            ins["dip_len"] = 32
            if b % 2 == 0:   # half the batches share one address pair: one huge bucket
                ins["sip"] = 0x0A000001
                ins["dip"] = 0x0B000001
            ins["id"] = np.arange(next_id, next_id + len(ins), dtype=np.uint32)
            ins["priority"] = rng.integers(0, 100_000, len(ins))
            next_id += len(ins)
            T.tang_insert(rs, ins)
            all_rules = np.concatenate([all_rules, ins])
        wild = synth.make_rules(50, seed=77, ordering="literal")
        wild["sip_len"] = 0
        wild["dip_len"] = 8
        wild["id"] = np.arange(next_id, next_id + 50, dtype=np.uint32)
        wild["priority"] = rng.integers(0, 100_000, 50)
        T.tang_insert(rs, wild)
        all_rules = np.concatenate([all_rules, wild])
        assert T.tang_ruleset_num_tuples(rs) == 2
        pk = synth.make_packets(all_rules, 40_000, seed=5, frac_in=0.9)
        pk[:2000]["sip"] = 0x0A000001
        pk[:2000]["dip"] = 0x0B000001
        want = orc.classify(all_rules, pk)
        assert np.array_equal(classify_dev(rs, pk), want)
        dels = all_rules["id"][rng.choice(len(all_rules), 5000, replace=False)]
        T.tang_delete(rs, dels)
        lm = ~np.isin(all_rules["id"], dels)
        assert np.array_equal(classify_dev(rs, pk), orc.classify(all_rules, pk, live=lm))
    finally:
        T.tang_ruleset_destroy(rs)


def test_update_rounds_at_512k_sampled():
    """The 512k-rule ruleset of the update workload: 3 rounds of 100 inserts + 100 deletes,
    each followed by a 1M-header lookup from the live rules; a seeded 5,000-header sample
    of every round equals the oracle's re-scan, and every answer contains its header."""
    torch_cuda()
    cfg = synth.CONFIGS["c4_512k_updates"]
    rules = synth.make_rules(cfg["n_rules"], seed=cfg["seed"], ordering="specificity")
    rs = T.tang_ruleset_create(0, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        Ws, bs = train.random_weights(C, 256, seed=3)
        T.tang_model_load(rs, Ws, bs, "bf16")
        all_rules = rules.copy()
        live = set(int(i) for i in rules["id"])
        for rd, (ins, dels) in enumerate(synth.make_update_stream(rules, 3, 100, seed=cfg["seed"] + 2,
                                                                  prio_range=len(rules))):
            T.tang_insert(rs, ins)
            T.tang_delete(rs, dels)
            all_rules = np.concatenate([all_rules, ins])
            live |= set(int(i) for i in ins["id"])
            live -= set(int(i) for i in dels)
            lm = _live_mask(all_rules, live)
            pk = synth.make_packets(all_rules[lm], cfg["n_pkts"], seed=rd, frac_in=cfg["frac_in"])
            got = classify_dev(rs, pk)
            samp = np.random.default_rng(rd).choice(len(pk), 5000, replace=False)
            assert np.array_equal(got[samp], orc.classify(all_rules, pk[samp], live=lm)), rd
            by_id = {int(r["id"]): k for k, r in enumerate(all_rules)}
            for k in samp[:300]:
                assert orc.rule_matches(all_rules[by_id[int(got[k])]], pk[k])
    finally:
        T.tang_ruleset_destroy(rs)
