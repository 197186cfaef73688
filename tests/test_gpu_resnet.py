"""The residual predictor (Sec. 6.1 with Eq. 1 blocks, Sec. 6.2 input) on MFMA against the
float64 oracle, and classification with it loaded (still bit-exact).

Tolerances, from the arithmetic. Every MFMA layer sums K = 512 products in FP32, so an
unrounded logit differs from the float64 value by at most about 4 K u m per layer
(u = 2^-24, m = the magnitude |W| |a| + |b| propagated by ``resnet_abs_forward``). BF16
rounding of a layer's output happens on both sides with the same rule, but when the FP32
and float64 values straddle a rounding boundary the two roundings differ by one BF16 unit
(2^-7 relative at most), which later layers carry to the logits scaled by at most m.

* Permutation blocks (w1 = w2 = P, zero biases) make every block exact on both sides
  (a block computes relu(P P x + x): one product per output, a sum of two BF16 values,
  the same rounding), so only the input layer (7 FP32 terms) and the output layer can
  differ: logits must meet 4 K u m, except on headers with an input-layer value within its
  FP32 error of a BF16 rounding boundary (one division and seven FMAs: at most about 4 u
  times the sum of the terms' magnitudes; 6 u is used),
  which get one unit more. A transposed operand, a wrong row, a lost residual or a
  chunk-boundary slip breaks the identity.
* Random weights: through 14 layers the |W| |a| magnitudes grow about 18x per layer, so
  a rigorous bound no longer bites. The test checks the error against each header's logit
  scale (max |logit|): rounding-boundary disagreements move a logit by about 2^-8 of a
  typical activation's size per affected layer, so the median relative error must stay
  below 2^-9 and the 99th percentile below 2^-6; and the top candidate must equal the
  oracle's wherever the top-two margin exceeds 2^-4 of the scale.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2601_03187_amd import synth
from paper_2601_03187_amd import tang as T
from tests._gpu import classify_dev, mlp_dev, torch_cuda

pytestmark = pytest.mark.gpu

W = 512
U = 2.0 ** -24


def _random_model(C, n_blocks, rng, scale=1.0):
    Ws = [rng.normal(0, 2.0 * scale, (W, 7))]
    bs = [rng.normal(0, 0.1 * scale, W)]
    for _ in range(2 * n_blocks):
        Ws.append(rng.normal(0, scale / np.sqrt(W), (W, W)))
        bs.append(rng.normal(0, 0.05 * scale, W))
    Ws.append(rng.normal(0, scale / np.sqrt(W), (C, W)))
    bs.append(rng.normal(0, 0.05 * scale, C))
    return [w.astype(np.float32) for w in Ws], [b.astype(np.float32) for b in bs]


def _near_boundary(pre, e):
    """Pre-activations whose ReLU-then-BF16 value could change under a perturbation of +-e
    (a value clipped to 0 either way is not near one)."""
    return orc.bf16_round(np.maximum(pre + e, 0)) != orc.bf16_round(np.maximum(pre - e, 0))


def _ruleset(n=1500, seed=61, wide=False):
    rules = synth.make_rules(n, seed=seed, wide=wide)
    rs = T.tang_ruleset_create(0, rules)
    return rules, rs, T.tang_ruleset_num_tuples(rs)


def test_permutation_blocks_exact_across_chunks():
    """70,001 headers (two workspace passes of 65,536, the second ragged), 2 blocks; the
    oracle on every header of a window around the chunk boundary and a seeded sample."""
    torch_cuda()
    rules, rs, C = _ruleset()
    try:
        rng = np.random.default_rng(7)
        Ws, bs = _random_model(C, 2, rng)
        P = np.eye(W, dtype=np.float32)[rng.permutation(W)]
        for k in range(1, 5):
            Ws[k] = P
            bs[k] = np.zeros(W, np.float32)
        T.tang_model_load_resnet(rs, Ws, bs, "bf16", topk=2)
        hdr = synth.make_packets(rules, 70_001, seed=62, frac_in=0.7)
        logits, cand = mlp_dev(rs, hdr, C, topk=2)
        rows = np.unique(np.concatenate([np.arange(65_520, 65_560),
                                         np.random.default_rng(8).choice(len(hdr), 600, replace=False)]))
        S = orc.segments(hdr[rows])
        want = orc.resnet_forward(S, Ws, bs, "bf16")
        mag = orc.resnet_abs_forward(S, Ws, bs)[-1]
        pre = S @ Ws[0].astype(np.float64).T + bs[0]
        e0 = 6 * U * (np.abs(S) @ np.abs(Ws[0].astype(np.float64)).T + np.abs(bs[0]))
        flip = _near_boundary(pre, e0).any(axis=1)
        tight = 4 * W * U * mag + 1e-30
        err = np.abs(logits[rows].astype(np.float64) - want)
        assert (err[~flip] <= tight[~flip]).all(), float((err / mag)[~flip].max())
        assert (err <= tight + 2.0 ** -7 * mag).all()
        assert flip.mean() < 0.5  # most headers get the tight check
        assert (cand < C).all() and (cand[:, 0] != cand[:, 1]).all()
    finally:
        T.tang_ruleset_destroy(rs)


@pytest.mark.parametrize("n_blocks,wide", [(1, False), (6, False), (2, True)])
def test_random_weights_within_bound_and_candidates(n_blocks, wide):
    """The paper's depth (6 blocks) and a single block, random weights; and a 144-tuple
    ruleset (several 64-class output blocks with a running top-k)."""
    torch_cuda()
    rules, rs, C = _ruleset(seed=63, wide=wide)
    assert C > 128 if wide else C <= 32
    try:
        Ws, bs = _random_model(C, n_blocks, np.random.default_rng(10 + n_blocks))
        T.tang_model_load_resnet(rs, Ws, bs, "bf16", topk=1)
        hdr = synth.make_packets(rules, 4099, seed=64, frac_in=0.7)
        logits, cand = mlp_dev(rs, hdr, C, topk=1)
        S = orc.segments(hdr)
        want = orc.resnet_forward(S, Ws, bs, "bf16")
        scale = np.abs(want).max(axis=1)
        rel = (np.abs(logits.astype(np.float64) - want).max(axis=1)) / scale
        assert np.isfinite(logits).all()
        assert np.median(rel) <= 2.0 ** -9 and np.percentile(rel, 99) <= 2.0 ** -6, \
            (float(np.median(rel)), float(np.percentile(rel, 99)), float(rel.max()))
        srt = np.sort(want, axis=1)
        clear = (srt[:, -1] - srt[:, -2]) > 2.0 ** -4 * scale
        assert clear.mean() > 0.3
        assert np.array_equal(cand[clear, 0], orc.topk(want, 1)[clear, 0])
    finally:
        T.tang_ruleset_destroy(rs)


def test_classify_with_residual_model_is_exact():
    """Rule ids do not depend on the predictor: with the residual model loaded (top-1 and
    top-2) every answer equals the oracle's."""
    torch_cuda()
    cfg = synth.CONFIGS["c1_1k"]
    rules = synth.make_rules(cfg["n_rules"], seed=cfg["seed"])
    hdr = synth.make_packets(rules, cfg["n_pkts"], seed=cfg["seed"] + 1, frac_in=cfg["frac_in"])
    want = orc.classify(rules, hdr)
    rs = T.tang_ruleset_create(0, rules)
    try:
        C = T.tang_ruleset_num_tuples(rs)
        Ws, bs = _random_model(C, 6, np.random.default_rng(21))
        for k in (1, 2):
            T.tang_model_load_resnet(rs, Ws, bs, "bf16", topk=k)
            assert np.array_equal(classify_dev(rs, hdr), want), k
    finally:
        T.tang_ruleset_destroy(rs)


def test_residual_model_validation():
    torch_cuda()
    rules, rs, C = _ruleset(500, seed=65)
    try:
        Ws, bs = _random_model(C, 1, np.random.default_rng(1))
        for args, kw in [((Ws, bs, "fp32"), {}),
                         ((Ws[:-1] + [Ws[-1][:-1]], bs[:-1] + [bs[-1][:-1]], "bf16"), {}),
                         ((Ws, bs, "bf16"), {"topk": 5})]:
            with pytest.raises(T.TangError) as e:
                T.tang_model_load_resnet(rs, *args, **kw)
            assert e.value.name == "EINVAL"
        narrow = [Ws[0][:256]] + [w[:256, :256] for w in Ws[1:3]] + [Ws[3][:, :256]]
        with pytest.raises(T.TangError):
            T.tang_model_load_resnet(rs, narrow, [bs[0][:256], bs[1][:256], bs[2][:256], bs[3]], "bf16")
    finally:
        T.tang_ruleset_destroy(rs)
