"""GPU parity: every rule id from the HIP path equals the linear-scan oracle's, bit for
bit, on the worked example, on exhaustive tiny universes, and on the benchmark
workloads (full answers at sizes the oracle finishes in seconds; sampled answers plus
invariants that hold at any size at the 512k-rule, 16M-header size)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2601_03187_amd import synth, train
from paper_2601_03187_amd import tang as T
from tests import _golden
from tests._gpu import classify_dev, keys_of, to_dev, torch_cuda

pytestmark = pytest.mark.gpu
NO = T.TANG_NO_MATCH


def _load(rs, Ws, bs, prec, topk=1, sc=None):
    T.tang_model_load(rs, Ws, bs, prec, topk=topk, act_scales=sc if prec == "fp8" else None)


def test_table1_grid_probe_all_and_with_models(golden_tab_rules):
    torch_cuda()
    g = golden_tab_rules
    rng = np.random.default_rng(3)
    pts, pk = _golden.grid_packets(rng, reps=4)
    want = np.array([NO if g["grid"][p] is None else int(g["grid"][p][1:]) for p in pts], dtype=np.uint32)
    rs = T.tang_ruleset_create(0, g["array"])
    try:
        assert np.array_equal(classify_dev(rs, pk), want)
        names = [t[0] for t in g["tuples"]]
        for rname, targets in g["conflict"].items():
            want_m = sum(1 << names.index(t) for t in targets)
            assert T.tang_ruleset_conflict_mask(rs, int(rname[1:])) == want_m, rname
        # every constant prediction (each tuple forced as argmax), all precisions
        for prec in ("fp32", "bf16", "fp8"):
            for winner in range(5):
                Ws, bs = train.constant_winner_weights(5, 128, winner)
                _load(rs, Ws, bs, prec, sc=[1.0, 1.0, 1.0])
                assert np.array_equal(classify_dev(rs, pk), want), (prec, winner)
        T.tang_model_unload(rs)
        # Sec. 4.3 / 5.2.1 insertions on the device
        for (name, prio, x, y, _) in g["inserts"]:
            T.tang_insert(rs, np.array([_golden.make_rule(name, prio, x, y)], dtype=synth.RULE_DTYPE))
        grid = dict(g["grid"])
        for (cx, cy, cell) in g["changes"]:
            grid[(cx, cy)] = cell
        want2 = np.array([NO if grid[p] is None else int(grid[p][1:]) for p in pts], dtype=np.uint32)
        assert np.array_equal(classify_dev(rs, pk), want2)
    finally:
        T.tang_ruleset_destroy(rs)


def test_exhaustive_restricted_universe():
    """Rules and packets confined to SIP/DIP top-3 bits, ports 0..7, protocol {6, 17}:
    all 8,192 packets of that universe against the oracle, probe-all and with models."""
    torch_cuda()
    rng = np.random.default_rng(11)
    n = 120
    r = np.zeros(n, dtype=synth.RULE_DTYPE)
    r["sip_len"] = rng.integers(1, 4, n)
    r["dip_len"] = rng.integers(0, 4, n)
    r["sip"] = (rng.integers(0, 8, n) << 29).astype(np.uint32)
    r["dip"] = (rng.integers(0, 8, n) << 29).astype(np.uint32)
    for f in ("sp", "dp"):
        a, b = rng.integers(0, 8, n), rng.integers(0, 8, n)
        wild = rng.random(n) < 0.15
        r[f + "_lo"] = np.where(wild, 0, np.minimum(a, b))
        r[f + "_hi"] = np.where(wild, 65535, np.maximum(a, b))
    pr = rng.choice([6, 17, 17, -1], n)
    r["proto"] = np.where(pr < 0, 0, pr)
    r["proto_mask"] = np.where(pr < 0, 0, 255)
    r["priority"] = rng.integers(0, 100, n)       # many ties -> id order decides
    r["id"] = rng.permutation(n).astype(np.uint32) + 5
    grid = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), np.arange(8), [6, 17],
                                indexing="ij"), -1).reshape(-1, 5)
    pk = np.zeros(len(grid), dtype=synth.HDR_DTYPE)
    pk["sip"] = (grid[:, 0] << 29).astype(np.uint32)
    pk["dip"] = (grid[:, 1] << 29).astype(np.uint32)
    pk["sp"], pk["dp"], pk["proto"] = grid[:, 2], grid[:, 3], grid[:, 4]
    want = orc.classify(r, pk)
    assert (want == NO).any() and (want != NO).any()
    rs = T.tang_ruleset_create(0, r)
    try:
        assert np.array_equal(classify_dev(rs, pk), want)
        C = T.tang_ruleset_num_tuples(rs)
        for seed in range(3):
            Ws, bs = train.random_weights(C, 128, seed=seed, scale=3.0)
            for prec in ("fp32", "bf16"):
                _load(rs, Ws, bs, prec, topk=1 + seed % 2)
                assert np.array_equal(classify_dev(rs, pk), want), (seed, prec)
    finally:
        T.tang_ruleset_destroy(rs)


def test_conflict_masks_equal_bruteforce():
    torch_cuda()
    rules = synth.make_rules(400, seed=21, ordering="specificity", mix=0.25)
    rules["priority"] = np.random.default_rng(0).integers(0, 50, len(rules))  # ties
    rt = orc.rule_tuples(rules)
    want = orc.conflict_masks(rules, rt)
    rs = T.tang_ruleset_create(0, rules)
    try:
        for k in range(len(rules)):
            assert T.tang_ruleset_rule_tuple(rs, int(rules[k]["id"])) == rt[k]
            assert T.tang_ruleset_conflict_mask(rs, int(rules[k]["id"])) == int(want[k]), k
    finally:
        T.tang_ruleset_destroy(rs)


@pytest.mark.parametrize("ordering", ["specificity", "literal"])
def test_c1_1k_rules_all_weights_identical(ordering):
    """1,024 rules, 10,000 headers (70% inside rules), 104 -> 128 -> 128 -> C: rule ids
    equal the oracle's with no model, trained, random, all-zero and adversarial weights."""
    torch_cuda()
    cfg = synth.CONFIGS["c1_1k"]
    rules = synth.make_rules(cfg["n_rules"], seed=cfg["seed"], ordering=ordering)
    hdr = synth.make_packets(rules, cfg["n_pkts"], seed=cfg["seed"] + 1, frac_in=cfg["frac_in"])
    want = orc.classify(rules, hdr)
    rs = T.tang_ruleset_create(0, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        got, st = classify_dev(rs, hdr, stats=True)
        assert np.array_equal(got, want)
        assert st["packets"] == len(hdr) and st["fallbacks"] == len(hdr)
        Ws, bs, sc, acc = train.fit(rs, rules, hdr, 128, steps=2000, seed=1, device="cuda")
        models = {"trained": (Ws, bs), "random": train.random_weights(C, 128, seed=2),
                  "zero": train.constant_winner_weights(C, 128, 0)}
        # adversarial: always predict the tuple holding the fewest answers
        lab = train.tuple_labels(rs, rules, want)
        worst = int(np.argmin(np.bincount(lab[lab >= 0], minlength=C)))
        models["adversarial"] = train.constant_winner_weights(C, 128, worst)
        for name, (W, b) in models.items():
            for prec in ("fp32", "bf16", "fp8"):
                for k in (1, 2):
                    _load(rs, W, b, prec, topk=k, sc=sc)
                    got, st = classify_dev(rs, hdr, stats=True)
                    assert np.array_equal(got, want), (name, prec, k)
        _load(rs, Ws, bs, "fp32")
        _, st = classify_dev(rs, hdr, stats=True)
        assert st["top1_hits"] > 0.5 * len(hdr), st  # the trained model mostly hits
    finally:
        T.tang_ruleset_destroy(rs)


_C2 = {}


def _c2_inputs():
    """The 64k-rule configuration at full size: rules, 1,000,000 headers, oracle answers."""
    if not _C2:
        cfg = synth.CONFIGS["c2_64k"]
        rules = synth.make_rules(cfg["n_rules"], seed=cfg["seed"], ordering="specificity", mix=cfg["mix"])
        hdr = synth.make_packets(rules, cfg["n_pkts"], seed=cfg["seed"] + 1, frac_in=cfg["frac_in"])
        _C2.update(rules=rules, hdr=hdr, want=orc.classify(rules, hdr))
    return _C2["rules"], _C2["hdr"], _C2["want"]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_c2_64k_rules_mix(prec):
    """65,536 rules with the 25% wildcard-heavy mix, 104 -> 256 -> 256 -> C; all
    1,000,000 headers of the configuration compared with the oracle."""
    torch_cuda()
    rules, hdr, want = _c2_inputs()
    rs = T.tang_ruleset_create(0, rules)
    try:
        assert np.array_equal(classify_dev(rs, hdr), want)
        Ws, bs, sc, acc = train.fit(rs, rules, hdr[:100_000], 256, steps=300, seed=3,
                                    rule_ids=want[:100_000], device="cuda")
        _load(rs, Ws, bs, prec)
        got, st = classify_dev(rs, hdr, stats=True)
        assert np.array_equal(got, want)
        assert st["packets"] == len(hdr) and st["probes"] <= 25 * len(hdr)
    finally:
        T.tang_ruleset_destroy(rs)


def test_chunked_two_stream_classify_equals_oracle():
    """A batch of at least two 2^21-header chunks with a model is classified chunk by
    chunk, the searches on the ruleset's own stream: the 1,000,000 headers of the 64k
    configuration tiled to 4,194,304 + 777 (a half chunk first and last, two ragged
    chunks between), every answer
    compared with the oracle's, on a side stream, twice in a row, for top-1 and top-2."""
    torch = torch_cuda()
    rules, hdr, want = _c2_inputs()
    reps = (2 * (1 << 21) + 777 + len(hdr) - 1) // len(hdr)
    big = np.concatenate([hdr] * reps)[: 2 * (1 << 21) + 777]
    big_want = np.concatenate([want] * reps)[: len(big)]
    rs = T.tang_ruleset_create(0, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        Ws, bs = train.random_weights(C, 256, seed=9)
        d_hdr = to_dev(big)
        d_out = torch.empty(len(big), dtype=torch.int32, device="cuda")
        side = torch.cuda.Stream()
        for topk in (1, 2):
            T.tang_model_load(rs, Ws, bs, "bf16", topk=topk)
            for _ in range(2):
                d_out.fill_(-7)
                torch.cuda.synchronize()
                T.tang_classify(rs, d_hdr, d_out, len(big), side)
                side.synchronize()
                assert np.array_equal(d_out.cpu().numpy().view(np.uint32), big_want), topk
    finally:
        T.tang_ruleset_destroy(rs)


def _c3_sampled(ordering, precs, sample_seed):
    """512k rules in the given order, 16,777,216 Zipf headers, in the launch shape the
    benchmark times (chunked over two streams for BF16 / FP8): every answer's key is <=
    the key of the rule the header was drawn from (an answer at least as good exists),
    every answer is a rule, the answer rule contains the header on a sample, and a seeded
    sample of 20,000 answers equals the oracle's. The same answers in every precision."""
    torch = torch_cuda()
    cfg = synth.CONFIGS["c3_512k"]
    rules = synth.make_rules(cfg["n_rules"], seed=cfg["seed"], ordering=ordering)
    assert np.array_equal(rules["id"], np.arange(len(rules)))  # id == index below
    hdr, src = synth.make_packets(rules, cfg["n_pkts"], seed=cfg["seed"] + 1,
                                  frac_in=cfg["frac_in"], zipf_s=cfg["zipf"], return_src=True)
    rs = T.tang_ruleset_create(0, rules)
    try:
        samp = np.random.default_rng(sample_seed).choice(len(hdr), 20_000, replace=False)
        want = orc.classify(rules, hdr[samp])
        Ws, bs, sc, acc = train.fit(rs, rules, hdr[:200_000], 256, steps=200, seed=4, device="cuda")
        first = None
        bound = keys_of(rules, rules["id"][src])
        for prec in precs:
            print(f"c3 {ordering} {prec}: {len(hdr)} headers", flush=True)
            _load(rs, Ws, bs, prec, sc=sc)
            got = classify_dev(rs, hdr)
            assert np.array_equal(got[samp], want), prec
            assert (got != NO).all()
            assert (keys_of(rules, got) <= bound).all()
            for k in samp[:200]:
                assert orc.rule_matches(rules[int(got[k])], hdr[k])
            if first is None:
                first = got
            else:
                assert np.array_equal(got, first), prec
        del torch
    finally:
        T.tang_ruleset_destroy(rs)


def test_c3_512k_rules_16m_headers_sampled():
    """The benchmark workload (specificity order) in BF16, FP8 and FP32."""
    _c3_sampled("specificity", ("bf16", "fp8", "fp32"), 5)


def test_c3_512k_literal_order_16m_headers_sampled():
    """The same 512k-rule generator in literal order (catch-all rules early shadow most
    later rules: long certification, many tuples per header), BF16 and FP32."""
    _c3_sampled("literal", ("bf16", "fp32"), 6)


def test_empty_and_ragged_batches():
    torch_cuda()
    rules = synth.make_rules(2000, seed=31)
    rs = T.tang_ruleset_create(0, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        Ws, bs = train.random_weights(C, 256, seed=3)
        _load(rs, Ws, bs, "bf16", topk=3)
        assert len(classify_dev(rs, np.zeros(0, dtype=synth.HDR_DTYPE))) == 0
        for n in (1, 15, 16, 17, 255, 257, 511, 4097, 33333):
            hdr = synth.make_packets(rules, n, seed=n, frac_in=0.6)
            assert np.array_equal(classify_dev(rs, hdr), orc.classify(rules, hdr)), n
    finally:
        T.tang_ruleset_destroy(rs)


def test_binding_refuses_buffers_shorter_than_n():
    """A wrong n from Python raises before any kernel runs; the right n classifies."""
    torch = torch_cuda()
    rules = synth.make_rules(500, seed=33)
    hdr = synth.make_packets(rules, 100, seed=34, frac_in=0.7)
    rs = T.tang_ruleset_create(0, rules)
    try:
        d_hdr = to_dev(hdr)
        d_out = torch.full((100,), -7, dtype=torch.int32, device="cuda")
        s = torch.cuda.current_stream()
        for args in [(d_hdr, d_out, 101), (d_hdr, d_out[:99], 100), (d_hdr, d_out[::2], 50)]:
            with pytest.raises(ValueError):
                T.tang_classify(rs, *args, s)
        torch.cuda.synchronize()
        assert (d_out.cpu().numpy() == -7).all()
        T.tang_classify(rs, d_hdr, d_out, 100, s)
        torch.cuda.synchronize()
        assert np.array_equal(d_out.cpu().numpy().view(np.uint32), orc.classify(rules, hdr))
        Ws, bs = train.random_weights(T.tang_ruleset_num_tuples(rs), 128, seed=1)
        _load(rs, Ws, bs, "bf16", topk=2)
        cand = torch.empty(150, dtype=torch.int16, device="cuda")   # needs 100 x 2
        with pytest.raises(ValueError):
            T.tang_mlp_forward(rs, d_hdr, 100, None, cand, s)
    finally:
        T.tang_ruleset_destroy(rs)


def test_empty_ruleset_answers_no_match():
    torch_cuda()
    rs = T.tang_ruleset_create(0, np.zeros(0, dtype=synth.RULE_DTYPE))
    try:
        hdr = synth.make_packets(np.zeros(0, dtype=synth.RULE_DTYPE), 1000, seed=1, frac_in=0.0)
        assert (classify_dev(rs, hdr) == NO).all()
    finally:
        T.tang_ruleset_destroy(rs)


def test_split_buckets_build_and_updates():
    """Thousands of rules under one (SIP, DIP) prefix pair: the bucket is kept as four
    sub-lists (exact DP, exact SP, exact protocol, rest). Answers equal the oracle's at
    build, after inserts and deletes into the sub-lists, and after a second bucket grows
    past the split threshold through inserts."""
    torch_cuda()
    rng = np.random.default_rng(8)
    rules = synth.make_rules(6000, seed=61, ordering="literal")
    rules["sip"], rules["sip_len"] = 0x0A000000, 8
    rules["dip"], rules["dip_len"] = 0, 0
    rules["priority"] = rng.integers(0, 3000, len(rules))       # ties -> ids decide
    others = synth.make_rules(3000, seed=62, ordering="specificity")
    others["id"] += 100_000
    others["priority"] += 1_000
    allr = np.concatenate([rules, others])
    pk = synth.make_packets(allr, 60_000, seed=63, frac_in=0.9)
    pk["sip"][:30_000] = (pk["sip"][:30_000] & 0x00FFFFFF) | 0x0A000000  # aim at the big bucket
    pk["proto"][:5000] = rng.choice([6, 17, 1, 141, 0], 5000)
    rs = T.tang_ruleset_create(0, allr)
    try:
        got, st = classify_dev(rs, pk, stats=True)
        assert np.array_equal(got, orc.classify(allr, pk))
        assert st["records"] < 60 * len(pk), st    # no header walks the whole bucket
        ins = synth.make_rules(500, seed=64, ordering="literal")
        ins["sip"], ins["sip_len"] = 0x0A000000, 8
        ins["dip"], ins["dip_len"] = 0, 0
        ins["id"] = np.arange(200_000, 200_500, dtype=np.uint32)
        ins["priority"] = rng.integers(0, 3000, 500)
        grow = synth.make_rules(40, seed=65, ordering="literal")   # a second bucket grows past 32
        grow["sip"], grow["sip_len"] = 0xC0A80000, 16
        grow["dip"], grow["dip_len"] = 0x0A0A0A00, 24
        grow["id"] = np.arange(300_000, 300_040, dtype=np.uint32)
        T.tang_insert(rs, ins)
        T.tang_insert(rs, grow)
        dels = rng.choice(rules["id"], 800, replace=False)
        T.tang_delete(rs, dels)
        allr2 = np.concatenate([allr, ins, grow])
        live = ~np.isin(allr2["id"], dels)
        pk2 = synth.make_packets(allr2[live], 60_000, seed=66, frac_in=0.9)
        pk2["sip"][:20_000] = (pk2["sip"][:20_000] & 0x00FFFFFF) | 0x0A000000
        pk2["sip"][20_000:25_000] = (pk2["sip"][20_000:25_000] & 0xFFFF) | 0xC0A80000
        pk2["dip"][20_000:25_000] = (pk2["dip"][20_000:25_000] & 0xFF) | 0x0A0A0A00
        assert np.array_equal(classify_dev(rs, pk2), orc.classify(allr2, pk2, live=live))
    finally:
        T.tang_ruleset_destroy(rs)
