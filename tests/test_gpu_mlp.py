"""Predictor on MFMA against the fp64 oracle MLP (Sec. 6.1, plain form).

Tolerance, derived from the arithmetic: every layer sums at most K = 104 + 2H products
in FP32, so with unit roundoff u = 2^-24 the accumulated error of a logit is bounded by
about K u times its magnitude m = |W3|(|W2|(|W1| x + |b1|) + |b2|) + |b3|; the test
allows 4 K u m ("tight"). BF16 / FP8 layer inputs are rounded on both sides with the
same rule, but an FP32 value and its fp64 counterpart can fall on different sides of a
rounding boundary, moving that input by one unit in the last place (2^-7 relative for
BF16, 2^-3 for FP8); the rigorous bound adds that ("loose"), and since such straddles
are rare, at least 99% of the logits must still meet the tight bound.
Where the tuple choice (an integer) depends on floating point, candidates are compared
only on rows whose top-two margin exceeds twice the tight bound.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2601_03187_amd import synth, train
from paper_2601_03187_amd import tang as T
from tests._gpu import mlp_dev, torch_cuda

pytestmark = pytest.mark.gpu

ULP_REL = {"fp32": 0.0, "bf16": 2.0 ** -7, "fp8": 2.0 ** -3}


def _hidden_amax(X, Ws, bs):
    h = X
    out = [1.0]
    for l in range(2):
        h = np.maximum(h @ Ws[l].astype(np.float64).T + bs[l], 0)
        out.append(float(h.max()) / 448.0)
    return out


@pytest.mark.parametrize("wide", [False, True, "all"])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("hidden", [128, 256])
def test_logits_and_candidates_vs_oracle(prec, hidden, wide):
    """wide: 144 tuples, so the output layer runs over several 32-class blocks with a
    running top-k; "all": every prefix length, 387 tuples (16-bit candidates)."""
    torch_cuda()
    rules = synth.make_rules(3000, seed=41, wide=wide is True, all_lengths=wide == "all")
    hdr = synth.make_packets(rules, 3001, seed=42, frac_in=0.7)  # ragged: not a tile multiple
    rs = T.tang_ruleset_create(0, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        Ws, bs = train.random_weights(C, hidden, seed=hidden + len(prec))
        X = orc.feature_bits(hdr)
        sc = _hidden_amax(X, Ws, bs)
        T.tang_model_load(rs, Ws, bs, prec, topk=2, act_scales=sc if prec == "fp8" else None)
        logits, cand = mlp_dev(rs, hdr, C, topk=2)
        want = orc.mlp_forward(X, Ws, bs, prec, act_scales=sc)
        mag = orc.mlp_abs_forward(X, Ws, bs)[-1]
        K = 104 + 2 * hidden
        tight = 4 * K * 2.0 ** -24 * mag + 1e-30
        loose = tight + 2 * ULP_REL[prec] * mag
        err = np.abs(logits.astype(np.float64) - want)
        assert np.isfinite(logits).all()
        assert (err <= loose).all(), float((err / mag).max())
        frac_tight = float((err <= tight).mean())
        assert frac_tight >= (1.0 if prec == "fp32" else 0.99), frac_tight
        # candidates: valid, distinct, and equal to the oracle's where the margin is clear
        assert (cand < C).all() and (cand[:, 0] != cand[:, 1]).all()
        srt = np.sort(want, axis=1)
        # on every row the first candidate is a maximum up to the logits' error: its oracle
        # score is within twice the loose bound of the oracle's best
        rows = np.arange(len(hdr))
        assert (want[rows, cand[:, 0]] >= srt[:, -1] - 2 * loose.max(axis=1)).all()
        margin = srt[:, -1] - srt[:, -2]
        rows_ok = (err <= tight).all(axis=1) & (margin > 2 * tight.max(axis=1))
        top = orc.topk(want, 2)
        # enough rows with a clear winner to make the check bite (144 classes crowd the top)
        assert rows_ok.mean() > (0.05 if wide else 0.25)
        assert np.array_equal(cand[rows_ok, 0], top[rows_ok, 0])
        third = np.sort(want, axis=1)[:, -3]
        rows2 = rows_ok & ((srt[:, -2] - third) > 2 * tight.max(axis=1))
        assert np.array_equal(cand[rows2, 1], top[rows2, 1])
    finally:
        T.tang_ruleset_destroy(rs)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("wide", [False, True])
def test_all_equal_scores_pick_lowest_indices(prec, wide):
    """Ties go to the lower tuple index, also across the 32-class blocks of a 144-tuple
    output layer; NaN scores (a NaN bias) still yield valid, distinct candidates."""
    torch_cuda()
    rules = synth.make_rules(1500 if wide else 500, seed=43, wide=wide)
    hdr = synth.make_packets(rules, 100, seed=44, frac_in=0.5)
    rs = T.tang_ruleset_create(0, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        Ws, bs = train.constant_winner_weights(C, 128, 0)
        bs[2][:] = 0.0  # every score equal
        sc = [1, 1, 1] if prec == "fp8" else None
        for k in (1, 3, 4):
            T.tang_model_load(rs, Ws, bs, prec, topk=k, act_scales=sc)
            logits, cand = mlp_dev(rs, hdr, C, topk=k)
            assert (logits == 0).all()
            assert (cand == np.arange(k)).all(), k
        bs[2][C - 1] = 1.0          # one winner in the last block, the rest tie
        bs[2][C // 2] = 0.5
        T.tang_model_load(rs, Ws, bs, prec, topk=3, act_scales=sc)
        _, cand = mlp_dev(rs, hdr, C, topk=3)
        assert (cand == np.array([C - 1, C // 2, 0])).all()
        bs[2][:] = np.nan
        T.tang_model_load(rs, Ws, bs, prec, topk=2, act_scales=sc)
        _, cand = mlp_dev(rs, hdr, C, topk=2)
        assert (cand < C).all() and (cand[:, 0] != cand[:, 1]).all()
    finally:
        T.tang_ruleset_destroy(rs)


def test_model_load_validation():
    torch_cuda()
    rules = synth.make_rules(500, seed=45)
    rs = T.tang_ruleset_create(0, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        Ws, bs = train.random_weights(C, 128, seed=1)
        bad_out = [Ws[0], Ws[1], Ws[2][:-1]]
        for args, kw in [((bad_out, [bs[0], bs[1], bs[2][:-1]], "fp32"), {}),
                         ((Ws, bs, "fp8"), {}),                           # no scales
                         ((Ws, bs, "bf16"), {"act_scales": [1, 1, 1]}),   # scales not FP8
                         ((Ws, bs, "fp32"), {"topk": 5}),
                         ((Ws, bs, "fp8"), {"act_scales": [1, 0.0, 1]}),
                         # a requantisation factor beyond 2^100 between the hidden layers
                         ((Ws, bs, "fp8"), {"act_scales": [1, 1e30, 1e-8]})]:
            with pytest.raises(T.TangError) as e:
                T.tang_model_load(rs, *args, **kw)
            assert e.value.name == "EINVAL"
        W2, b2 = train.random_weights(C, 192, seed=1)
        with pytest.raises(T.TangError):
            T.tang_model_load(rs, W2, b2, "fp32")
    finally:
        T.tang_ruleset_destroy(rs)
