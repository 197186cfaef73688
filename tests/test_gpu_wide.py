"""Wide tuple spaces (more than 32 tuples; the paper's rulesets have 31 to 391): eight
conflict-mask words per rule, tuple indices past 32 in candidates, prefix prunes and
filter sweeps over all eight words. Every answer equals the oracle's linear scan."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2601_03187_amd import synth, train
from paper_2601_03187_amd import tang as T
from tests._gpu import classify_dev, torch_cuda

pytestmark = pytest.mark.gpu


def test_wide_conflict_masks_equal_bruteforce():
    """1,500 rules over 144 tuples, priorities with ties: all eight words of every rule's
    mask equal the brute-force mask (bit t: a rule in tuple t precedes it and overlaps)."""
    torch_cuda()
    rules = synth.make_rules(1500, seed=71, wide=True)
    rules["priority"] = np.random.default_rng(0).integers(0, 100, len(rules))
    rt = orc.rule_tuples(rules)
    want = orc.conflict_masks(rules, rt)
    rs = T.tang_ruleset_create(0, rules)
    try:
        assert T.tang_ruleset_num_tuples(rs) == 144
        assert max(int(w) for w in want) >> 32  # some mask reaches past word 0
        for k in range(len(rules)):
            assert T.tang_ruleset_rule_tuple(rs, int(rules[k]["id"])) == rt[k]
            assert T.tang_ruleset_conflict_mask(rs, int(rules[k]["id"])) == int(want[k]), k
    finally:
        T.tang_ruleset_destroy(rs)


def test_wide_classify_no_model_and_every_predictor():
    """20,000 rules over 144 tuples, 100,003 headers (80% inside rules): rule ids equal the
    oracle's with no model, the plain MLP (128 and 256 wide, FP32 / BF16 / FP8, top-1 and
    top-4, trained and random weights) and the residual model."""
    torch_cuda()
    rules = synth.make_rules(20_000, seed=72, wide=True)
    hdr = synth.make_packets(rules, 100_003, seed=73, frac_in=0.8)
    want = orc.classify(rules, hdr)
    rs = T.tang_ruleset_create(0, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        assert C == 144
        got, st = classify_dev(rs, hdr, stats=True)
        assert np.array_equal(got, want)
        assert st["no_match"] == int((want == orc.NO_MATCH).sum())
        for hidden in (128, 256):
            Ws, bs, sc, acc = train.fit(rs, rules, hdr[:50_000], hidden, steps=300, seed=hidden,
                                        rule_ids=want[:50_000], device="cuda")
            models = {"trained": (Ws, bs), "random": train.random_weights(C, hidden, seed=5)}
            for name, (W, b) in models.items():
                for prec in ("fp32", "bf16", "fp8"):
                    for k in (1, 4):
                        T.tang_model_load(rs, W, b, prec, topk=k,
                                          act_scales=sc if prec == "fp8" else None)
                        assert np.array_equal(classify_dev(rs, hdr), want), (hidden, name, prec, k)
        rng = np.random.default_rng(9)
        Wr = [rng.normal(0, 2.0, (512, 7))] + [rng.normal(0, 1 / np.sqrt(512), (512, 512)) for _ in range(4)]
        Wr.append(rng.normal(0, 1 / np.sqrt(512), (C, 512)))
        br = [rng.normal(0, 0.05, w.shape[0]) for w in Wr]
        for k in (1, 2):
            T.tang_model_load_resnet(rs, [w.astype(np.float32) for w in Wr],
                                     [b.astype(np.float32) for b in br], "bf16", topk=k)
            assert np.array_equal(classify_dev(rs, hdr), want), ("resnet", k)
    finally:
        T.tang_ruleset_destroy(rs)


def test_wide_updates_and_appended_tuples():
    """A 121-tuple ruleset (no zero-length prefixes): update rounds, some inserts with
    lengths no tuple has (restricted insertion), then signatures no tuple dominates (new
    tuples 121, 122, beyond the first mask word's range); answers equal the oracle's after
    every batch and conflict masks stay supersets of the brute-force ones."""
    torch_cuda()
    rules = synth.make_rules(20_000, seed=74, wide=True)
    rules = rules[(rules["sip_len"] > 0) & (rules["dip_len"] > 0)]
    rs = T.tang_ruleset_create(0, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        assert C == 121
        hdr0 = synth.make_packets(rules, 40_000, seed=2, frac_in=0.8)
        Ws, bs, sc, acc = train.fit(rs, rules, hdr0, 256, steps=200, seed=3, device="cuda")
        T.tang_model_load(rs, Ws, bs, "bf16", topk=2)
        all_rules = rules.copy()
        live = set(int(i) for i in rules["id"])
        ups = synth.make_update_stream(rules, rounds=4, per_round=200, seed=75,
                                       prio_range=len(rules))
        rng = np.random.default_rng(76)
        for rd, (ins, dels) in enumerate(ups):
            ins["sip_len"] = np.maximum(ins["sip_len"], 8)   # (0, d) would append a tuple
            ins["dip_len"] = np.maximum(ins["dip_len"], 8)
            odd = rng.random(len(ins)) < 0.3
            ins["sip_len"][odd] = rng.choice([21, 27, 31], odd.sum())
            ins["sip"][odd] &= np.uint32(0xFFFFFFF0)
            if rd == 3:  # two signatures below every tuple: appended as tuples C, C + 1
                ins["sip_len"][:40] = 0
                ins["dip_len"][:20] = 4
                ins["dip_len"][20:40] = 0
            T.tang_insert(rs, ins)
            T.tang_delete(rs, dels)
            all_rules = np.concatenate([all_rules, ins])
            live |= set(int(i) for i in ins["id"])
            live -= set(int(i) for i in dels)
            lm = np.isin(all_rules["id"], np.fromiter(live, dtype=np.uint32))
            assert T.tang_ruleset_num_tuples(rs) == (C + 2 if rd == 3 else C)
            pk = synth.make_packets(all_rules[lm], 60_000, seed=200 + rd, frac_in=0.8)
            want = orc.classify(all_rules, pk, live=lm)
            assert np.array_equal(classify_dev(rs, pk), want), rd
        assert T.tang_ruleset_tuple(rs, C) == (0, 4) and T.tang_ruleset_tuple(rs, C + 1) == (0, 0)
        small = all_rules[lm]
        tup = np.array([T.tang_ruleset_rule_tuple(rs, int(i)) for i in small["id"]])
        assert (tup == C + 1).sum() > 0
        key = small["priority"].astype(np.uint64) << np.uint64(32) | small["id"].astype(np.uint64)
        for k in rng.choice(len(small), 40, replace=False):
            m = T.tang_ruleset_conflict_mask(rs, int(small[k]["id"]))
            prior = np.flatnonzero(key < key[k])
            need = 0
            for j in prior:
                if orc.boxes_intersect(small[j], small[k]):
                    need |= 1 << int(tup[j])
            assert m & need == need, (k, hex(m), hex(need))
    finally:
        T.tang_ruleset_destroy(rs)


def test_wide_chunked_classify():
    """A 144-tuple ruleset through the chunked classify (two 2^21-header chunks and a
    ragged third, each chunk's search on the ruleset's stream behind the next chunk's
    model): every answer equals the oracle's, with a trained and with a random model,
    BF16 top-1 and FP8 top-2."""
    torch = torch_cuda()
    rules = synth.make_rules(20_000, seed=78, wide=True)
    hdr = synth.make_packets(rules, 100_000, seed=79, frac_in=0.8)
    want = orc.classify(rules, hdr)
    n = 2 * (1 << 21) + 333
    reps = (n + len(hdr) - 1) // len(hdr)
    big = np.concatenate([hdr] * reps)[:n]
    big_want = np.concatenate([want] * reps)[:n]
    rs = T.tang_ruleset_create(0, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        Ws, bs, sc, acc = train.fit(rs, rules, hdr[:50_000], 256, steps=300, seed=4,
                                    rule_ids=want[:50_000], device="cuda")
        d_hdr = torch.from_numpy(big.view(np.uint8).reshape(-1).copy()).cuda()
        d_out = torch.empty(n, dtype=torch.int32, device="cuda")
        for name, (W, b) in {"trained": (Ws, bs), "random": train.random_weights(C, 256, seed=6)}.items():
            for prec, k in (("bf16", 1), ("fp8", 2)):
                T.tang_model_load(rs, W, b, prec, topk=k, act_scales=sc if prec == "fp8" else None)
                d_out.fill_(-7)
                T.tang_classify(rs, d_hdr, d_out, n, torch.cuda.current_stream())
                torch.cuda.synchronize()
                assert np.array_equal(d_out.cpu().numpy().view(np.uint32), big_want), (name, prec)
    finally:
        T.tang_ruleset_destroy(rs)
