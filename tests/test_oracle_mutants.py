"""The oracle's pins bite: a copy of each pinned function with one plausible mistake
planted in it (on the CPU) fails at least one pin.

Each copy below is first checked to equal the oracle when no mistake is planted, so the
mistakes are planted in the oracle's own arithmetic and not in a different function.
The pins come from tests/test_oracle_pins.py and tests/test_oracle_resnet_pins.py.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from tests.test_oracle_pins import mlp_quant_cases, run_quant_case
from tests.test_oracle_resnet_pins import WIDTH_TWO_MAGS, width_two_network

# --- mlp_forward ------------------------------------------------------------------------

MLP_MISTAKES = ["bf16_no_weight_round", "bf16_no_input_round", "bf16_round_bias",
                "bf16_round_logits", "fp8_no_weight_round", "fp8_no_act_round",
                "fp8_no_saturate", "fp8_scales_layer0", "fp8_amax_scale_hidden",
                "fp8_deq_weight_only",
                "fp8_deq_act_only", "relu_on_logits", "no_bias", "no_relu"]


def _e4m3_unsaturated(x):
    """E4M3 rounding that lets magnitudes beyond 448 through unrounded."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(np.abs(x) > orc.E4M3_MAX, x, orc.e4m3_round(x))


def _mlp_copy(x, Ws, bs, precision="fp32", act_scales=None, mistake=None):
    a = np.asarray(x, dtype=np.float64)
    L = len(Ws)
    for l in range(L):
        W = np.asarray(Ws[l], dtype=np.float64)
        b = np.asarray(bs[l], dtype=np.float64)
        if mistake == "no_bias":
            b = np.zeros_like(b)
        if precision == "fp32":
            z = a @ W.T + b
        elif precision == "bf16":
            qa = a if mistake == "bf16_no_input_round" else orc.bf16_round(a)
            qw = W if mistake == "bf16_no_weight_round" else orc.bf16_round(W)
            qb = orc.bf16_round(b) if mistake == "bf16_round_bias" else b
            z = qa @ qw.T + qb
        elif precision == "fp8":
            rnd = _e4m3_unsaturated if mistake == "fp8_no_saturate" else orc.e4m3_round
            s_a = (float(np.float32(act_scales[l])) if (l > 0 or mistake == "fp8_scales_layer0")
                   else 1.0)
            if l < L - 1 and mistake != "fp8_amax_scale_hidden":
                s_w = orc.fp8_hidden_weight_scale(W, s_a, float(np.float32(act_scales[l + 1])))
            else:
                s_w = orc.fp8_weight_scale(W)
            inv_a = float(np.float32(1.0 / s_a))
            inv_w = float(np.float32(1.0 / s_w))
            qa = a * inv_a if mistake == "fp8_no_act_round" else rnd(a * inv_a)
            qw = W * inv_w if mistake == "fp8_no_weight_round" else rnd(W * inv_w)
            if mistake == "fp8_deq_weight_only":
                deq = float(np.float32(s_w))
            elif mistake == "fp8_deq_act_only":
                deq = float(np.float32(s_a))
            else:
                deq = float(np.float32(np.float32(s_a) * np.float32(s_w)))
            z = (qa @ qw.T) * deq + b
        else:
            raise ValueError(precision)
        last = l == L - 1
        if mistake == "no_relu" and not last:
            a = z
        elif mistake == "relu_on_logits" or not last:
            a = np.maximum(z, 0.0)
        else:
            a = z
    if precision == "bf16" and mistake == "bf16_round_logits":
        a = orc.bf16_round(a)
    return a


def _mlp_pins_hold(fwd) -> bool:
    """The hand-computed quantisation cases and the FP32 closed forms of the pins."""
    x, cases = mlp_quant_cases()
    for c in cases:
        if not np.allclose(run_quant_case(fwd, x, c), c[5], rtol=1e-6, atol=0):
            return False
    # one-hot input selects a weight column and ReLU clips (FP32)
    W1 = np.zeros((3, 104)); W1[:, 7] = [2.0, -1.0, 0.5]
    xo = np.zeros((1, 104)); xo[0, 7] = 1.0
    if fwd(xo, [W1, np.eye(3), np.eye(3)], [np.zeros(3)] * 3).tolist() != [[2.0, 0.0, 0.5]]:
        return False
    # zero weights give the output bias; a negative output bias stays negative
    bs = [np.array([1.0, -2.0]), np.array([0.5, 0.5]), np.array([-1.5, 2.5])]
    Ws = [np.zeros((2, 104)), np.zeros((2, 2)), np.zeros((2, 2))]
    if fwd(xo, Ws, bs).tolist() != [[-1.5, 2.5]]:
        return False
    # a negative hidden pre-activation is clipped before the next layer
    Ws = [np.zeros((1, 104)), np.ones((1, 1)), np.ones((1, 1))]
    if fwd(xo, Ws, [np.array([-4.0]), np.zeros(1), np.zeros(1)]).tolist() != [[0.0]]:
        return False
    return True


def test_mlp_copy_equals_oracle_without_mistake():
    rng = np.random.default_rng(5)
    dims = [104, 24, 24, 7]
    Ws = [rng.normal(0, 0.3, (dims[i + 1], dims[i])) for i in range(3)]
    bs = [rng.normal(0, 0.3, dims[i + 1]) for i in range(3)]
    x = rng.integers(0, 2, size=(40, 104)).astype(float)
    sc = [1.0, 0.01, 0.02]
    for prec in ("fp32", "bf16", "fp8"):
        want = orc.mlp_forward(x, Ws, bs, prec, act_scales=sc)
        assert np.array_equal(_mlp_copy(x, Ws, bs, prec, act_scales=sc), want), prec
    assert _mlp_pins_hold(orc.mlp_forward)
    assert _mlp_pins_hold(_mlp_copy)


@pytest.mark.parametrize("mistake", MLP_MISTAKES)
def test_mlp_pins_catch(mistake):
    fwd = lambda *a, **k: _mlp_copy(*a, **k, mistake=mistake)  # noqa: E731
    assert not _mlp_pins_hold(fwd), mistake


# --- mlp_abs_forward --------------------------------------------------------------------

ABS_MISTAKES = ["signed_weights", "no_bias", "forward_activations", "no_abs_input",
                "abs_of_sum"]


def _mlp_abs_copy(x, Ws, bs, mistake=None):
    a = np.asarray(x, dtype=np.float64)
    if mistake != "no_abs_input":
        a = np.abs(a)
    mags = []
    for W, b in zip(Ws, bs):
        W = np.asarray(W, np.float64)
        b = np.asarray(b, np.float64)
        if mistake == "signed_weights":
            m = a @ W.T + np.abs(b)
        elif mistake == "no_bias":
            m = a @ np.abs(W).T
        elif mistake == "abs_of_sum":
            m = np.abs(a @ W.T + b)
        else:
            m = a @ np.abs(W).T + np.abs(b)
        mags.append(m)
        a = np.maximum(a @ W.T + b, 0.0) if mistake == "forward_activations" else m
    return mags


def _mlp_abs_pins_hold(absf) -> bool:
    x = np.array([[1.0, -1.0]])
    Ws = [np.array([[1.0, -2.0], [-1.0, 0.0]]), np.array([[1.0, -1.0]]), np.array([[-2.0], [0.5]])]
    bs = [np.array([0.5, -3.0]), np.array([-1.0]), np.array([0.25, -0.25])]
    if [m.tolist() for m in absf(x, Ws, bs)] != [[[3.5, 4.0]], [[8.5]], [[17.25, 4.5]]]:
        return False
    rng = np.random.default_rng(11)
    dims = [104, 10, 9, 6]
    Ws = [rng.random((dims[i + 1], dims[i])) for i in range(3)]
    bs = [rng.random(dims[i + 1]) for i in range(3)]
    x = rng.integers(0, 2, size=(8, 104)).astype(float)
    return bool(np.allclose(absf(x, Ws, bs)[-1], orc.mlp_forward(x, Ws, bs), rtol=1e-13, atol=0))


def test_mlp_abs_copy_equals_oracle_without_mistake():
    rng = np.random.default_rng(6)
    Ws = [rng.normal(size=(5, 104)), rng.normal(size=(5, 5)), rng.normal(size=(3, 5))]
    bs = [rng.normal(size=5), rng.normal(size=5), rng.normal(size=3)]
    x = rng.integers(0, 2, size=(9, 104)).astype(float)
    for a, b in zip(_mlp_abs_copy(x, Ws, bs), orc.mlp_abs_forward(x, Ws, bs)):
        assert np.array_equal(a, b)
    assert _mlp_abs_pins_hold(orc.mlp_abs_forward)


@pytest.mark.parametrize("mistake", ABS_MISTAKES)
def test_mlp_abs_pins_catch(mistake):
    assert not _mlp_abs_pins_hold(lambda *a: _mlp_abs_copy(*a, mistake=mistake)), mistake


# --- resnet_abs_forward -----------------------------------------------------------------

RES_ABS_MISTAKES = ["no_residual", "signed_weights", "no_bias", "residual_from_h"]


def _resnet_abs_copy(s, Ws, bs, mistake=None):
    f = lambda a: np.abs(np.asarray(a, dtype=np.float64))  # noqa: E731
    sw = (lambda a: np.asarray(a, dtype=np.float64)) if mistake == "signed_weights" else f
    fb = (lambda a: 0.0 * np.asarray(a, dtype=np.float64)) if mistake == "no_bias" else f
    a = f(s) @ sw(Ws[0]).T + fb(bs[0])
    mags = [a]
    for k in range((len(Ws) - 2) // 2):
        h = a @ sw(Ws[1 + 2 * k]).T + fb(bs[1 + 2 * k])
        res = 0.0 if mistake == "no_residual" else (h if mistake == "residual_from_h" else a)
        a = h @ sw(Ws[2 + 2 * k]).T + fb(bs[2 + 2 * k]) + res
        mags += [h, a]
    mags.append(a @ sw(Ws[-1]).T + fb(bs[-1]))
    return mags


def _resnet_abs_pins_hold(absf) -> bool:
    s, Ws, bs = width_two_network()
    return [m.tolist() for m in absf(s, Ws, bs)] == WIDTH_TWO_MAGS


def test_resnet_abs_copy_equals_oracle_without_mistake():
    rng = np.random.default_rng(7)
    Ws = [rng.normal(size=(6, 7))] + [rng.normal(size=(6, 6)) for _ in range(4)] + \
        [rng.normal(size=(3, 6))]
    bs = [rng.normal(size=w.shape[0]) for w in Ws]
    s = rng.random((5, 7))
    for a, b in zip(_resnet_abs_copy(s, Ws, bs), orc.resnet_abs_forward(s, Ws, bs)):
        assert np.array_equal(a, b)
    assert _resnet_abs_pins_hold(orc.resnet_abs_forward)


@pytest.mark.parametrize("mistake", RES_ABS_MISTAKES)
def test_resnet_abs_pins_catch(mistake):
    assert not _resnet_abs_pins_hold(lambda *a: _resnet_abs_copy(*a, mistake=mistake)), mistake
