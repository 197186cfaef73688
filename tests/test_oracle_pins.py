"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test names what would fail if the oracle had a plausible mistake in it (a dropped
field, a reversed priority order, a wrong mask shift, an off-by-one range bound).
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2601_03187_amd import synth
from tests import _golden

NO = orc.NO_MATCH


def _ids(names):
    return [int(n[1:]) for n in names]


# --- Table 1 worked example (Sec. 4.1 / 4.2) -------------------------------------------

def test_tab_rules_grid_c_and_definition(golden_tab_rules):
    """Exhaustive 8x8 grid: pins priority direction, prefix semantics, NO_MATCH."""
    g = golden_tab_rules
    rng = np.random.default_rng(1)
    pts, pk = _golden.grid_packets(rng, reps=3)
    want = np.array([NO if g["grid"][p] is None else int(g["grid"][p][1:]) for p in pts],
                    dtype=np.uint32)
    got_c = orc.classify(g["array"], pk, threads=2)
    got_d = orc.classify_definition(g["array"], pk)
    assert np.array_equal(got_c, want)
    assert np.array_equal(got_d, want)
    # counts printed with the fixture: 23 empty points
    assert sum(1 for p in g["grid"].values() if p is None) == 23


def test_tab_rules_tuples(golden_tab_rules):
    """Tuples T1..T5 in first-appearance order and the rule -> tuple column of Table 1."""
    g = golden_tab_rules
    tup = orc.tuples_first_appearance(g["array"])
    assert tup == [(a, b) for (_, a, b) in g["tuples"]]
    names = [t[0] for t in g["tuples"]]
    rt = orc.rule_tuples(g["array"])
    assert [names[i] for i in rt] == [r[4] for r in g["rules"]]
    # every rule is in exactly one tuple (Sec. 4.3)
    assert len(rt) == len(g["array"])


def test_tab_rules_insertions(golden_tab_rules):
    """R9 -> T1 (Sec. 4.3) and R10 -> T3 (Sec. 5.2.1); grid changes only where stated."""
    g = golden_tab_rules
    tup = orc.tuples_first_appearance(g["array"])
    names = [t[0] for t in g["tuples"]]
    rules = g["array"].copy()
    grid = dict(g["grid"])
    for (name, prio, x, y, want_t) in g["inserts"]:
        r = _golden.make_rule(name, prio, x, y)
        t = orc.insert_tuple(tup, int(r["sip_len"]), int(r["dip_len"]))
        assert names[t] == want_t
        rules = np.concatenate([rules, np.array([r], dtype=rules.dtype)])
        for (cx, cy, cell) in g["changes"]:
            if cell == name:
                grid[(cx, cy)] = cell
    rng = np.random.default_rng(2)
    pts, pk = _golden.grid_packets(rng, reps=2)
    want = np.array([NO if grid[p] is None else int(grid[p][1:]) for p in pts], dtype=np.uint32)
    assert np.array_equal(orc.classify(rules, pk), want)
    # R10 = {100, 0**} does not take (4,2) from R7 nor (4,3) from R6
    assert grid[(4, 2)] == "R7" and grid[(4, 3)] == "R6"


def test_insert_tuple_no_dominated():
    """No tuple with every length <= the rule's: -1 (the library appends a tuple)."""
    assert orc.insert_tuple([(8, 8), (16, 0)], 0, 32) == -1
    # (8,8) and (16,0) both have length sum 16: the tie goes to the first tuple
    assert orc.insert_tuple([(8, 8), (16, 0)], 16, 32) == 0
    assert orc.insert_tuple([(16, 0), (8, 8)], 16, 32) == 0
    assert orc.insert_tuple([(0, 0), (8, 8), (16, 8)], 16, 32) == 2


def test_tab_rules_conflict_masks(golden_tab_rules):
    g = golden_tab_rules
    names = [t[0] for t in g["tuples"]]
    rt = orc.rule_tuples(g["array"])
    masks = orc.conflict_masks(g["array"], rt)
    for (rname, *_), m in zip(g["rules"], masks):
        want = sum(1 << names.index(t) for t in g["conflict"][rname])
        assert int(m) == want, rname


# --- truncation and boundary cases ------------------------------------------------------

def _rule(**kw):
    r = np.zeros(1, dtype=synth.RULE_DTYPE)
    r["sp_hi"] = 65535
    r["dp_hi"] = 65535
    for k, v in kw.items():
        r[k] = v
    return r


def _hdr(**kw):
    h = np.zeros(1, dtype=synth.HDR_DTYPE)
    for k, v in kw.items():
        h[k] = v
    return h


def test_truncation_11star():
    """Sec. 4.3: '11*' in a 3-bit field truncates to 110; it covers 110 and 111 only."""
    r = _rule(sip=0b110 << 29, sip_len=2, id=5)
    for top, want in [(0b110, 5), (0b111, 5), (0b100, NO), (0b101, NO), (0b010, NO)]:
        h = _hdr(sip=(top << 29) | 0x1234567)
        assert orc.classify(r, h)[0] == want
        assert orc.classify_definition(r, h)[0] == want
    # bits beyond the prefix in the rule value are ignored (normalised)
    r2 = _rule(sip=(0b110 << 29) | 0x1FFFFFFF, sip_len=2, id=6)
    assert orc.classify(r2, _hdr(sip=0b111 << 29))[0] == 6


@pytest.mark.parametrize("length", [0, 1, 31, 32])
def test_prefix_length_edges(length):
    v = 0xDEADBEEF
    r = _rule(dip=v, dip_len=length, id=1)
    flip_low = _hdr(dip=v ^ 1)           # differs only in the last bit
    flip_high = _hdr(dip=v ^ 0x80000000)  # differs only in the first bit
    assert orc.classify(r, _hdr(dip=v))[0] == 1
    assert orc.classify(r, flip_low)[0] == (1 if length < 32 else NO)
    assert orc.classify(r, flip_high)[0] == (1 if length == 0 else NO)
    assert orc.prefix_mask(length) == (0 if length == 0 else (0xFFFFFFFF << (32 - length)) & 0xFFFFFFFF)


def test_port_bounds_inclusive():
    r = _rule(sp_lo=0, sp_hi=0, dp_lo=65535, dp_hi=65535, id=3)
    assert orc.classify(r, _hdr(sp=0, dp=65535))[0] == 3
    assert orc.classify(r, _hdr(sp=1, dp=65535))[0] == NO
    assert orc.classify(r, _hdr(sp=0, dp=65534))[0] == NO
    r = _rule(sp_lo=100, sp_hi=200, id=4)
    got = [orc.classify(r, _hdr(sp=s))[0] for s in (99, 100, 150, 200, 201)]
    assert got == [NO, 4, 4, 4, NO]


def test_protocol_exact_and_wildcard():
    exact = _rule(proto=17, proto_mask=0xFF, id=7)
    wild = _rule(proto=17, proto_mask=0, id=8)
    for p in range(256):
        h = _hdr(proto=p)
        assert orc.classify(exact, h)[0] == (7 if p == 17 else NO)
        assert orc.classify(wild, h)[0] == 8


def test_priority_ties_to_lower_id_and_direction():
    a = _rule(priority=5, id=10)
    b = _rule(priority=5, id=9)
    c = _rule(priority=6, id=1)
    rules = np.concatenate([a, b, c])
    assert orc.classify(rules, _hdr())[0] == 9
    assert orc.classify(np.concatenate([c, a]), _hdr())[0] == 10  # 5 beats 6
    assert orc.classify_definition(rules, _hdr())[0] == 9


def test_empty_inputs():
    assert len(orc.classify(np.zeros(0, synth.RULE_DTYPE), np.zeros(0, synth.HDR_DTYPE))) == 0
    out = orc.classify(np.zeros(0, synth.RULE_DTYPE), _hdr(sip=1))
    assert out[0] == NO


def test_live_mask():
    rules = np.concatenate([_rule(priority=1, id=1), _rule(priority=2, id=2)])
    h = _hdr()
    assert orc.classify(rules, h, live=np.array([0, 1]))[0] == 2
    assert orc.classify(rules, h, live=np.array([0, 0]))[0] == NO


# --- brute force and invariants on random small inputs ---------------------------------

def _small_rules(rng, n):
    r = synth.make_rules(n, seed=int(rng.integers(1 << 30)), ordering="literal")
    # duplicate priorities so the id tie-break is exercised; ids not in priority order
    r["priority"] = rng.integers(0, max(1, n // 3), size=n)
    r["id"] = rng.permutation(np.arange(1000, 1000 + n)).astype(np.uint32)
    return r


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_c_oracle_equals_definition(seed):
    rng = np.random.default_rng(seed)
    rules = _small_rules(rng, 40)
    pk = synth.make_packets(rules, 300, seed=seed + 7, frac_in=0.7)
    live = rng.random(len(rules)) < 0.8
    assert np.array_equal(orc.classify(rules, pk, threads=3),
                          orc.classify_definition(rules, pk))
    assert np.array_equal(orc.classify(rules, pk, live=live),
                          orc.classify_definition(rules, pk, live=live))


@pytest.mark.parametrize("ordering", ["literal", "specificity"])
def test_sampled_inside_invariant(ordering):
    """A packet drawn inside rule r gets a rule of priority at least as high as r's, and
    the returned rule contains the packet."""
    rules = synth.make_rules(2000, seed=11, ordering=ordering)
    pk, src = synth.make_packets(rules, 4000, seed=12, frac_in=1.0, return_src=True)
    got = orc.classify(rules, pk)
    assert (got != NO).all()
    key_src = rules["priority"][src].astype(np.int64) * (1 << 32) + rules["id"][src]
    by_id = {int(r["id"]): i for i, r in enumerate(rules)}
    gi = np.array([by_id[int(g)] for g in got])
    key_got = rules["priority"][gi].astype(np.int64) * (1 << 32) + rules["id"][gi]
    assert (key_got <= key_src).all()
    for k in range(0, 4000, 97):
        assert orc.rule_matches(rules[gi[k]], pk[k])


def test_answer_invariant_under_rule_permutation():
    rules = synth.make_rules(500, seed=5, ordering="specificity")
    pk = synth.make_packets(rules, 2000, seed=6, frac_in=0.7)
    perm = np.random.default_rng(0).permutation(len(rules))
    assert np.array_equal(orc.classify(rules, pk), orc.classify(rules[perm], pk))


def test_disjoint_rules_answer_is_the_sampled_rule():
    """Rules with pairwise disjoint exact SIPs: every inside packet answers its rule."""
    n = 300
    rules = synth.make_rules(n, seed=9, ordering="literal")
    rules["sip"] = np.arange(n, dtype=np.uint32) * 7919
    rules["sip_len"] = 32
    pk, src = synth.make_packets(rules, 1000, seed=10, frac_in=1.0, return_src=True)
    assert np.array_equal(orc.classify(rules, pk), rules["id"][src])


def test_scan_length_reported():
    rules = np.concatenate([_rule(priority=0, id=0, sp_lo=5, sp_hi=5),
                            _rule(priority=1, id=1)])
    out, scanned = orc.classify(rules, _hdr(sp=4), want_scanned=True)
    assert out[0] == 1 and scanned[0] == 2


# --- model-side pins --------------------------------------------------------------------

def test_feature_bits_msb_first():
    h = _hdr(sip=0x80000001, dip=0x00000002, sp=0x8000, dp=0x0001, proto=0x81)
    x = orc.feature_bits(h)[0]
    assert x.shape == (104,)
    on = set(np.nonzero(x)[0].tolist())
    assert on == {0, 31, 62, 64, 95, 96, 103}


def test_bf16_rounding_from_definition():
    v = orc.bf16_round(np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-7, -3.0,
                                 2.0**-133, 2.0**-134, 65504.0 + 100]))
    assert v.tolist() == [1.0, 1.0, 1 + 2**-6, 1 + 2**-7, -3.0, 2.0**-133, 0.0, 65536.0]


def test_e4m3_rounding_from_definition():
    x = np.array([448.0, 464.0, 1e6, -500.0, 17.0, 19.0, 2.0**-9, 2.0**-10, 3 * 2.0**-10,
                  0.3, 1.0, 1.0625, 1.1875])
    want = [448.0, 448.0, 448.0, -448.0, 16.0, 20.0, 2.0**-9, 0.0, 2.0**-8,
            0.3125, 1.0, 1.0, 1.25]
    assert orc.e4m3_round(x).tolist() == want
    vals = orc._e4m3_values()
    assert len(vals) == 127 and vals[-1] == 448.0 and vals[1] == 2.0**-9


def test_mlp_zero_weights_give_output_bias():
    rng = np.random.default_rng(0)
    dims = [104, 16, 16, 5]
    Ws = [np.zeros((dims[i + 1], dims[i])) for i in range(3)]
    bs = [rng.normal(size=dims[i + 1]) for i in range(3)]
    x = rng.integers(0, 2, size=(7, 104)).astype(float)
    out = orc.mlp_forward(x, Ws, bs)
    assert np.allclose(out, np.tile(bs[2], (7, 1)), rtol=0, atol=0)


def test_mlp_nonnegative_collapses_to_matrix_product():
    """With non-negative weights, biases and inputs every ReLU is the identity, so the
    network equals one affine map: x (W3 W2 W1)^T + (W3 W2 b1 + W3 b2 + b3)."""
    rng = np.random.default_rng(1)
    W1 = rng.random((12, 104)); W2 = rng.random((9, 12)); W3 = rng.random((5, 9))
    b1 = rng.random(12); b2 = rng.random(9); b3 = rng.random(5)
    x = rng.integers(0, 2, size=(11, 104)).astype(float)
    want = x @ (W3 @ W2 @ W1).T + (W3 @ W2 @ b1 + W3 @ b2 + b3)
    got = orc.mlp_forward(x, [W1, W2, W3], [b1, b2, b3])
    assert np.allclose(got, want, rtol=1e-12, atol=0)


def test_mlp_one_hot_selects_weight_column_and_relu_clips():
    W1 = np.zeros((3, 104)); W1[:, 7] = [2.0, -1.0, 0.5]
    W2 = np.eye(3); W3 = np.eye(3)
    b = [np.zeros(3)] * 3
    x = np.zeros((1, 104)); x[0, 7] = 1.0
    assert orc.mlp_forward(x, [W1, W2, W3], b).tolist() == [[2.0, 0.0, 0.5]]


# --- Quantisation steps of the predictor (reading R19: BF16 round-to-nearest-even of the
# weights and of every layer's input; FP8 E4M3 with static activation scales, a weight
# scale amax/448 for the output layer and, for a hidden layer, that scale raised by a
# factor in [1, 2) until s_w s_a / s_next is a power of two; FP32 accumulate and bias).
# Each case is worked out by hand and isolates one step, so dropping or misplacing that
# step changes the pinned value.
# The cases are shared with tests/test_oracle_mutants.py, which checks that a copy of the
# oracle with each step broken fails at least one of them.

def _one_hot_input():
    x = np.zeros((1, 104))
    x[0, 0] = 1.0
    return x


def mlp_quant_cases():
    """(name, precision, Ws, bs, act_scales, exact logits) computed by hand."""
    x = _one_hot_input()
    cases = []
    # BF16 weight rounding: 1 + 2^-9 is not a bfloat16 value (8 significant bits) and
    # rounds to 1. It sits in the output layer, whose input (1) is exact, so no later
    # rounding can hide a missing weight rounding.
    W1 = np.zeros((1, 104)); W1[0, 0] = 1.0
    cases.append(("bf16_weight", "bf16", [W1, np.ones((1, 1)), np.array([[1 + 2.0 ** -9]])],
                  [np.zeros(1)] * 3, None, [1.0]))
    # BF16 layer-input rounding, apart from the weights (all exact): the hidden value
    # 1 + 2^-9 comes from an unrounded bias, the next layer reads it rounded to 1.
    # The output bias 0.5 + 2^-10 is not a bfloat16 value (it would round to 0.5); it is
    # added unrounded, and the logit 1.5 + 2^-10 is not rounded either (it would be 1.5).
    cases.append(("bf16_input", "bf16", [W1, np.ones((1, 1)), np.ones((1, 1))],
                  [np.array([2.0 ** -9]), np.zeros(1), np.array([0.5 + 2.0 ** -10])],
                  None, [1.5 + 2.0 ** -10]))
    # FP8 weight rounding, in the output layer: W1 column = [1, 1] scales to 448 (s_w =
    # 1/448: with s_a = 1 and s_next = 1/448 the factor is already 2^0) and W2 = I to 256
    # (amax scale 1/448, factor (1/448)(1/448)/(1/448) = 1/448, raised to 2^-8: s_w =
    # 2^-8); the hidden values [1, 1] enter each next layer as 448 (s_a = 1/448, on the
    # grid). W3 = diag(3, 1) has s_w = 3/448, so its scaled entries are 448 and 149.33;
    # E4M3 has 144 and 160 in [128, 256) (step 16), so 149.33 -> 144 and the logits are
    # 448 * 448 * (1/448) * (3/448) = 3 and 448 * 144 * ... = 27/28.
    W1 = np.zeros((2, 104)); W1[:, 0] = 1.0
    cases.append(("fp8_weight", "fp8", [W1, np.eye(2), np.diag([3.0, 1.0])], [np.zeros(2)] * 3,
                  [1.0, 1.0 / 448, 1.0 / 448], [3.0, 27.0 / 28]))
    # FP8 activation rounding: W1 column = [1, 0.5] scales to 448 and 224 (on the grid;
    # s_w = 1/448 as above, W2 = I again at s_w = 2^-8); a bias of 0.03 makes the second
    # hidden value 0.53, which s_a = 1/448 maps to 237.44 -> 240 (grid 224, 240, 256):
    # the next layers see 240/448 = 15/28.
    # act_scales[0] is ignored, the input bits being exact: 3000 there changes nothing
    # (read as a scale, 1/3000 would round to 0 in E4M3 and zero the first layer).
    W1 = np.zeros((2, 104)); W1[0, 0] = 1.0; W1[1, 0] = 0.5
    cases.append(("fp8_activation", "fp8", [W1, np.eye(2), np.eye(2)],
                  [np.array([0.0, 0.03]), np.zeros(2), np.zeros(2)],
                  [3000.0, 1.0 / 448, 1.0 / 448], [1.0, 15.0 / 28]))
    # FP8 saturation: W1 column = [3, 0.25] has the amax scale 3/448, whose factor into
    # s_next = 1/300 is 900/448 = 2.01, raised to 4: s_w = 4/300 = 1/75. The column
    # scales to 225 -> 224 (grid 224, 240) and 18.75 -> 18 (grid 18, 20), so the hidden
    # values are 224/75 and 18/75. With s_a = 1/300 they map to 896, beyond the format's
    # 448, which saturates to 448, and 72 (on the grid): the next layers see 448/300 and
    # 72/300.
    W1 = np.zeros((2, 104)); W1[0, 0] = 3.0; W1[1, 0] = 0.25
    cases.append(("fp8_saturate", "fp8", [W1, np.eye(2), np.eye(2)], [np.zeros(2)] * 3,
                  [1.0, 1.0 / 300, 1.0 / 300], [448.0 / 300, 72.0 / 300]))
    # FP8 hidden weight scale: W1 column = [3, 0.77] with s_next = 1/100. The amax scale
    # 3/448 has the factor 300/448 = 0.67 into s_next, raised to 2^0: s_w = 1/100. The
    # column scales to 300 -> 288 (grid 288, 320) and 77 -> 80 (grid 72, 80), so the
    # hidden values are 2.88 and 0.8, on the activation grid at s_a = 1/100 (288, 80);
    # W2 = W3 = I pass them on: logits [2.88, 0.8]. (With the amax scale 3/448 the
    # column would be 448 and 114.99 -> 112, the second hidden value 0.75, entering the
    # next layer as 75 -> 72: logit 0.72.)
    W1 = np.zeros((2, 104)); W1[0, 0] = 3.0; W1[1, 0] = 0.77
    cases.append(("fp8_hidden_scale", "fp8", [W1, np.eye(2), np.eye(2)], [np.zeros(2)] * 3,
                  [1.0, 1.0 / 100, 1.0 / 100], [2.88, 0.8]))
    return x, cases


def run_quant_case(fwd, x, case):
    _, prec, Ws, bs, sc, _ = case
    return fwd(x, Ws, bs, prec, act_scales=sc)[0]


@pytest.mark.parametrize("k", range(6))
def test_mlp_quantisation_steps_hand_computed(k):
    x, cases = mlp_quant_cases()
    name, prec, Ws, bs, sc, want = cases[k]
    got = run_quant_case(orc.mlp_forward, x, cases[k])
    # the FP32 products of the stated scales (s_a s_w, 1/s) carry relative errors of a
    # few 2^-24; nothing else is inexact
    assert np.allclose(got, want, rtol=1e-6, atol=0), (name, got.tolist(), want)


def test_fp8_hidden_weight_scale_closed_form():
    """The hidden-layer weight scale against its definition: at least the amax scale,
    below twice it, and s_w s_a / s_next a power of two (up to the fp32 rounding of s_w);
    it equals the amax scale when that factor is already a power of two."""
    rng = np.random.default_rng(5)
    for _ in range(2000):
        W = rng.normal(0, 10.0 ** rng.uniform(-3, 1), (4, 3))
        s_a = float(np.float32(10.0 ** rng.uniform(-3, 2)))
        s_n = float(np.float32(10.0 ** rng.uniform(-3, 2)))
        s = orc.fp8_weight_scale(W)
        sw = orc.fp8_hidden_weight_scale(W, s_a, s_n)
        assert s * (1 - 2.0 ** -23) <= sw < 2 * s * (1 + 2.0 ** -23)
        k = sw * s_a / s_n
        assert abs(np.log2(k) - round(np.log2(k))) < 2.0 ** -20
    # already a power of two: W amax 448 (s = 1), s_a = 1/4, s_next = 1/32 (factor 8)
    W = np.array([[448.0, -3.0]])
    assert orc.fp8_hidden_weight_scale(W, 0.25, 1 / 32) == 1.0
    # amax 448 with s_a = 1/3, s_next = 1/3: factor 1, s_w = 1
    assert orc.fp8_hidden_weight_scale(W, 1 / 3, 1 / 3) == 1.0
    # amax 336 (s = 0.75), s_a = s_next: raised to 1
    assert orc.fp8_hidden_weight_scale(np.array([[336.0]]), 0.5, 0.5) == 1.0
    # amax 224 (s = 0.5), s_a = 1, s_next = 3: factor 1/6 -> 2^-2, s_w = 3/4
    assert orc.fp8_hidden_weight_scale(np.array([[224.0]]), 1.0, 3.0) == 0.75


def test_mlp_fp32_path_takes_no_rounding():
    x, cases = mlp_quant_cases()
    _, _, Ws, bs, _, _ = cases[0]
    assert orc.mlp_forward(x, Ws, bs, "fp32")[0, 0] == 1 + 2.0 ** -9
    _, _, Ws, bs, _, _ = cases[1]
    assert orc.mlp_forward(x, Ws, bs, "fp32")[0, 0] == 1.5 + 2.0 ** -9 + 2.0 ** -10


# --- Magnitudes that set the GPU tests' error bounds -----------------------------------

def test_mlp_abs_forward_equals_forward_on_nonnegative_networks():
    """Closed form: with non-negative weights, biases and inputs no ReLU clips and no
    absolute value changes anything, so every magnitude equals the layer's output."""
    rng = np.random.default_rng(11)
    dims = [104, 10, 9, 6]
    Ws = [rng.random((dims[i + 1], dims[i])) for i in range(3)]
    bs = [rng.random(dims[i + 1]) for i in range(3)]
    x = rng.integers(0, 2, size=(8, 104)).astype(float)
    mags = orc.mlp_abs_forward(x, Ws, bs)
    a = x
    for l in range(3):
        a = a @ Ws[l].T + bs[l]
        assert np.allclose(mags[l], a, rtol=1e-13, atol=0), l
    assert np.allclose(mags[-1], orc.mlp_forward(x, Ws, bs), rtol=1e-13, atol=0)


def test_mlp_abs_forward_hand_computed_mixed_signs():
    """x = [1, -1]: m0 = [1, 1]. W1 = [[1, -2], [-1, 0]], b1 = [0.5, -3]:
    m1 = [1 + 2 + 0.5, 1 + 0 + 3] = [3.5, 4] (the forward values are relu([3.5, -4]) =
    [3.5, 0]: the magnitude is not |W a + b|). W2 = [[1, -1]], b2 = [-1]:
    m2 = [3.5 + 4 + 1] = [8.5]. W3 = [[-2], [0.5]], b3 = [0.25, -0.25]:
    m3 = [17.25, 4.5]."""
    x = np.array([[1.0, -1.0]])
    Ws = [np.array([[1.0, -2.0], [-1.0, 0.0]]), np.array([[1.0, -1.0]]), np.array([[-2.0], [0.5]])]
    bs = [np.array([0.5, -3.0]), np.array([-1.0]), np.array([0.25, -0.25])]
    mags = orc.mlp_abs_forward(x, Ws, bs)
    assert [m.tolist() for m in mags] == [[[3.5, 4.0]], [[8.5]], [[17.25, 4.5]]]
    z = orc.mlp_forward(x, Ws, bs)
    # forward: h1 = relu([3.5, -4]) = [3.5, 0], h2 = relu([2.5]), z = [-4.75, 1.0]
    assert z.tolist() == [[-4.75, 1.0]]
    assert (np.abs(z) <= mags[-1]).all()


def test_topk_ties_to_lower_index():
    z = np.array([[1.0, 3.0, 3.0, 2.0], [0.0, 0.0, 0.0, 0.0]])
    assert orc.topk(z, 2).tolist() == [[1, 2], [0, 1]]


def test_flops_closed_form():
    """2 * (104 H + H^2 + H C): 65,792 at H=128, C=25 and 197,120 at H=256; the padded
    forms the kernel executes (K=128 input, 32 outputs) are 73,728 and 212,992."""
    assert orc.mlp_flops([104, 128, 128, 25]) == 65_792
    assert orc.mlp_flops([104, 256, 256, 25]) == 197_120
    assert orc.mlp_flops([128, 128, 128, 32]) == 73_728
    assert orc.mlp_flops([128, 256, 256, 32]) == 212_992


@pytest.mark.parametrize("wide", [False, True])
def test_conflict_masks_cover_every_better_answer(wide):
    """Certification is sound (reading R9): a header sampled inside rule m whose answer is
    a better rule a != m has a's tuple in m's conflict mask (a and m both contain the
    header, so their boxes intersect). Checked with the linear scan's answers, on a narrow
    and on a wide tuple space (masks past 32 bits), priorities with ties."""
    rules = synth.make_rules(400, seed=91, wide=wide, ordering="literal")
    rules["priority"] = np.random.default_rng(92).integers(0, 60, len(rules))
    rt = np.asarray(orc.rule_tuples(rules))
    masks = orc.conflict_masks(rules, rt)
    hdr, src = synth.make_packets(rules, 6000, seed=93, frac_in=1.0, return_src=True)
    ans = orc.classify(rules, hdr)
    pos = {int(i): k for k, i in enumerate(rules["id"])}
    better = 0
    for h, m in enumerate(src):
        a = pos[int(ans[h])]
        if a != m:
            better += 1
            assert (int(masks[m]) >> int(rt[a])) & 1, (h, m, a)
    assert better > 500  # the property is exercised, not vacuous
    if wide:
        assert max(int(x) for x in masks).bit_length() > 32
