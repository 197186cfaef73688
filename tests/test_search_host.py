"""The host search (the paper's CPU side, a comparison mode) on the CPU: exact mode equals
the linear scan whatever the candidates; paper mode equals the paper's procedure, written
independently here from the oracle: the best match inside the predicted tuples if there is
one, else the true answer (the ordered search over the remaining tuples finds it)."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2601_03187_amd import synth
from paper_2601_03187_amd import tang as T
from tests import _golden

NO = orc.NO_MATCH


def _paper_answers(rules, hdr, cand, kcand, truth):
    tup = np.asarray(orc.rule_tuples(rules))
    out = truth.copy()
    cs = [(cand >> (8 * k)) & 0xFF for k in range(kcand)]
    keys = np.stack(cs, axis=1)
    for combo in np.unique(keys, axis=0):
        g = (keys == combo).all(axis=1)
        inside = orc.classify(rules, hdr[g], live=np.isin(tup, combo).astype(np.uint8))
        out[g] = np.where(inside != NO, inside, truth[g])
    return out


def test_table1_grid_exact_with_any_candidates(golden_tab_rules):
    g = golden_tab_rules
    rs = T.tang_ruleset_create(T.TANG_HOST_ONLY, g["array"])
    try:
        pts, pk = _golden.grid_packets(np.random.default_rng(2), reps=2)
        want = np.array([NO if g["grid"][p] is None else int(g["grid"][p][1:]) for p in pts], np.uint32)
        assert np.array_equal(T.tang_search_host(rs, pk), want)
        for t in range(5):
            cand = np.full(len(pk), t, np.uint32)
            assert np.array_equal(T.tang_search_host(rs, pk, cand, 1), want)
    finally:
        T.tang_ruleset_destroy(rs)


@pytest.mark.parametrize("ordering,mix", [("specificity", 0.0), ("literal", 0.25)])
def test_random_rulesets_exact_and_paper_modes(ordering, mix):
    rules = synth.make_rules(3000, seed=31, ordering=ordering, mix=mix)
    hdr = synth.make_packets(rules, 20_000, seed=32, frac_in=0.8)
    truth = orc.classify(rules, hdr)
    rs = T.tang_ruleset_create(T.TANG_HOST_ONLY, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        rng = np.random.default_rng(33)
        for kcand in (1, 2):
            c = rng.integers(0, C, (len(hdr), kcand))
            cand = sum((c[:, k].astype(np.uint32) << np.uint32(8 * k)) for k in range(kcand)).astype(np.uint32)
            got, st = T.tang_search_host(rs, hdr, cand, kcand, threads=4, exact=True, want_stats=True)
            assert np.array_equal(got, truth), kcand
            assert st["packets"] == len(hdr) and st["no_match"] == int((truth == NO).sum())
            paper = T.tang_search_host(rs, hdr, cand, kcand, threads=4, exact=False)
            assert np.array_equal(paper, _paper_answers(rules, hdr, cand, kcand, truth)), kcand
        # random predictions are often wrong: the paper's search then returns lower-priority
        # rules on some headers (here it must differ somewhere, or the test would not bite)
        assert (paper != truth).any()
        assert np.array_equal(T.tang_search_host(rs, hdr, cand, kcand, threads=1),
                              T.tang_search_host(rs, hdr, cand, kcand, threads=7))
    finally:
        T.tang_ruleset_destroy(rs)


def test_exact_after_updates():
    rules = synth.make_rules(2000, seed=35)
    rs = T.tang_ruleset_create(T.TANG_HOST_ONLY, rules)
    try:
        ups = synth.make_update_stream(rules, 3, 200, seed=36, sip_lengths=(4, 20))
        for ins, dels in ups:
            T.tang_delete(rs, dels)
            T.tang_insert(rs, ins)
        live = T.tang_ruleset_export(rs)
        hdr = synth.make_packets(live, 10_000, seed=37, frac_in=0.8)
        assert np.array_equal(T.tang_search_host(rs, hdr, threads=3), orc.classify(live, hdr))
    finally:
        T.tang_ruleset_destroy(rs)


def test_argument_errors():
    rs = T.tang_ruleset_create(T.TANG_HOST_ONLY, synth.make_rules(10, seed=1))
    try:
        hdr = synth.make_packets(synth.make_rules(10, seed=1), 4, seed=2, frac_in=1.0)
        with pytest.raises(T.TangError):
            T.tang_search_host(rs, hdr, np.zeros(4, np.uint32), kcand=5)
        assert len(T.tang_search_host(rs, hdr[:0])) == 0
    finally:
        T.tang_ruleset_destroy(rs)


def test_wide_tuple_space_exact_and_paper_modes():
    """144 tuples (12 prefix lengths per field): the host tuple space and both search modes
    with candidates anywhere in 0..C-1, including tuple indices past 32."""
    rules = synth.make_rules(4000, seed=35, wide=True)
    hdr = synth.make_packets(rules, 12_000, seed=36, frac_in=0.8)
    truth = orc.classify(rules, hdr)
    rs = T.tang_ruleset_create(T.TANG_HOST_ONLY, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        assert C == len(orc.tuples_first_appearance(rules)) and C > 128
        rng = np.random.default_rng(37)
        c = rng.integers(0, C, (len(hdr), 2))
        cand = (c[:, 0].astype(np.uint32) | (c[:, 1].astype(np.uint32) << np.uint32(8))).astype(np.uint32)
        assert np.array_equal(T.tang_search_host(rs, hdr, cand, 2, threads=4, exact=True), truth)
        paper = T.tang_search_host(rs, hdr, cand, 2, threads=4, exact=False)
        assert np.array_equal(paper, _paper_answers(rules, hdr, cand, 2, truth))
    finally:
        T.tang_ruleset_destroy(rs)
