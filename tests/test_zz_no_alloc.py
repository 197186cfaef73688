"""tang_classify_host_noalloc (static staging, no device allocation) against
tang_classify_host on the same inputs: identical rule ids and statistics, on two calls in
a row (the second smaller, so stale staging from the first would show), with and
without a model, and the oracle as the final word. Sizes beyond the static staging are
refused before any device work."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2601_03187_amd import synth, train
from paper_2601_03187_amd import tang as T

pytestmark = pytest.mark.gpu


def _ruleset(n_rules, seed):
    rules = synth.make_rules(n_rules, seed=seed, ordering="specificity")
    return rules, T.tang_ruleset_create(0, rules)


@pytest.mark.parametrize("model", [None, "bf16"])
def test_noalloc_equals_classify_host_two_calls(model):
    rules, rs = _ruleset(4096, 1201)
    try:
        if model:
            C = T.tang_ruleset_num_tuples(rs)
            Ws, bs = train.random_weights(C, 256, seed=1202)
            T.tang_model_load(rs, Ws, bs, model, topk=2)
        # first call at the staging maximum, second one ragged and much smaller
        for n, seed in ((T.TANG_NOALLOC_MAX_HEADERS, 1203), (3001, 1204)):
            hdr = synth.make_packets(rules, n, seed=seed, frac_in=0.7)
            print(f"noalloc: model={model} n={n} seed={seed}", flush=True)
            want, st_want = T.tang_classify_host(rs, hdr, want_stats=True)
            got, st_got = T.tang_classify_host_noalloc(rs, hdr, want_stats=True)
            assert np.array_equal(got, want)
            assert st_got == st_want
            got2 = T.tang_classify_host_noalloc(rs, hdr)
            assert np.array_equal(got2, want)
            idx = np.random.default_rng(seed).choice(n, size=min(n, 3000), replace=False)
            assert np.array_equal(got[idx], orc.classify(rules, hdr[idx]))
    finally:
        T.tang_ruleset_destroy(rs)


def test_noalloc_two_rulesets_share_the_staging():
    rules_a, rs_a = _ruleset(2048, 1211)
    rules_b, rs_b = _ruleset(1024, 1212)
    try:
        ha = synth.make_packets(rules_a, 50000, seed=1213, frac_in=0.8)
        hb = synth.make_packets(rules_b, 777, seed=1214, frac_in=0.8)
        ga = T.tang_classify_host_noalloc(rs_a, ha)
        gb = T.tang_classify_host_noalloc(rs_b, hb)
        assert np.array_equal(ga, T.tang_classify_host(rs_a, ha))
        assert np.array_equal(gb, T.tang_classify_host(rs_b, hb))
        assert np.array_equal(gb, orc.classify(rules_b, hb))
    finally:
        T.tang_ruleset_destroy(rs_a)
        T.tang_ruleset_destroy(rs_b)


def test_noalloc_refuses_more_than_the_staging_and_takes_empty():
    rules, rs = _ruleset(256, 1221)
    try:
        hdr = np.zeros(T.TANG_NOALLOC_MAX_HEADERS + 1, dtype=synth.HDR_DTYPE)
        with pytest.raises(T.TangError) as ei:
            T.tang_classify_host_noalloc(rs, hdr)
        assert ei.value.code == -1 and "at most" in str(ei.value)
        assert len(T.tang_classify_host_noalloc(rs, hdr[:0])) == 0
    finally:
        T.tang_ruleset_destroy(rs)
