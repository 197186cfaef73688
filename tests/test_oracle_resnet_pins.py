"""Pins of the oracle's residual network (Sec. 6.1, Eq. 1; input format of Sec. 6.2).

Each case is fixed by hand or by a special case with a closed form, so that a plausible
mistake in the oracle fails one of them: a dropped residual term, the ReLU on the wrong
side of the sum, a transposed weight, a missing bias, a chunk out of order, a block
counted twice, or the residual taken before BF16 rounding.
"""
import numpy as np

from oracle import oracle as orc
from paper_2601_03187_amd import synth


def _model(width, n_blocks, C, rng, scale=0.2):
    Ws = [rng.normal(0, scale, (width, 7))]
    bs = [rng.normal(0, scale, width)]
    for _ in range(2 * n_blocks):
        Ws.append(rng.normal(0, scale / np.sqrt(width), (width, width)))
        bs.append(rng.normal(0, scale, width))
    Ws.append(rng.normal(0, scale, (C, width)))
    bs.append(rng.normal(0, scale, C))
    return Ws, bs


def test_segments_chunk_order_and_scale():
    """SIP 192.168.0.1, DIP 10.0.0.2, SP 443, DP 65535, PROTO 6 -> the seven chunks
    0xC0A8, 0x0001, 0x0A00, 0x0002, 443, 65535, 6, each over 65535."""
    p = np.zeros(1, dtype=synth.HDR_DTYPE)
    p["sip"], p["dip"], p["sp"], p["dp"], p["proto"] = 0xC0A80001, 0x0A000002, 443, 65535, 6
    want = np.array([[49320, 1, 2560, 2, 443, 65535, 6]]) / 65535.0
    assert np.array_equal(orc.segments(p), want)


def test_hand_computed_width_two_network():
    """Width 2, one block, three outputs, all values exact in BF16:
    a = relu(W_in s + b_in) = relu([2, -1 + 3]) = [2, 2];
    h = relu(W1 a + b1) = relu([2 + 2, -2 + 1]) = [4, 0];
    y = relu(W2 h + b2 + a) = relu([2 - 1 + 2, 4 - 0 + 2]) = [3, 6];
    z = W_out y + b_out = [3, 6, 3 - 6 + 10] = [3, 6, 7]."""
    s = np.zeros((1, 7))
    s[0, 0] = 1.0
    W_in = np.zeros((2, 7))
    W_in[0, 0], W_in[1, 0] = 2.0, -1.0
    b_in = np.array([0.0, 3.0])
    W1, b1 = np.array([[1.0, 1.0], [0.0, -1.0]]), np.array([0.0, 1.0])
    W2, b2 = np.array([[0.5, 0.0], [1.0, -1.0]]), np.array([-1.0, 0.0])
    Wo, bo = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, -1.0]]), np.array([0.0, 0.0, 10.0])
    for prec in ("fp32", "bf16"):
        z = orc.resnet_forward(s, [W_in, W1, W2, Wo], [b_in, b1, b2, bo], prec)
        assert np.array_equal(z, [[3.0, 6.0, 7.0]]), prec


def test_zero_blocks_collapse_to_two_layer_network():
    """With w1 = w2 = 0 and b1 = b2 = 0 a block maps x >= 0 to relu(x) = x, so any number
    of such blocks leaves W_out relu(W_in s + b_in) + b_out."""
    rng = np.random.default_rng(3)
    Ws, bs = _model(16, 3, 5, rng)
    for k in range(1, 7):
        Ws[k] = np.zeros_like(Ws[k])
        bs[k] = np.zeros_like(bs[k])
    s = rng.random((50, 7))
    want = np.maximum(s @ Ws[0].T + bs[0], 0) @ Ws[-1].T + bs[-1]
    assert np.allclose(orc.resnet_forward(s, Ws, bs, "fp32"), want, rtol=1e-13, atol=1e-13)


def test_identity_blocks_double_each_time():
    """With w1 = w2 = I and zero biases a block maps x >= 0 to relu(relu(x) + x) = 2x:
    k blocks scale the input layer's output by 2^k (exact in BF16 as well, so the BF16
    result is the rounded weights applied to 2^k times the rounded activations)."""
    rng = np.random.default_rng(4)
    width, C = 8, 3
    Ws, bs = _model(width, 4, C, rng)
    for k in range(1, 9):
        Ws[k] = np.eye(width)
        bs[k] = np.zeros(width)
    s = rng.random((40, 7))
    a0 = np.maximum(s @ Ws[0].T + bs[0], 0)
    assert np.allclose(orc.resnet_forward(s, Ws, bs, "fp32"), (16 * a0) @ Ws[-1].T + bs[-1],
                       rtol=1e-13, atol=1e-13)
    want16 = (16 * orc.bf16_round(a0)) @ orc.bf16_round(Ws[-1]).T + bs[-1]
    assert np.allclose(orc.resnet_forward(s, Ws, bs, "bf16"), want16, rtol=1e-13, atol=1e-13)


def test_bf16_residual_is_the_rounded_block_input():
    """Width 1, one block with w1 = w2 = 0: the block returns its (rounded) input. An
    input-layer output of 1 + 2^-9 is not a BF16 value and rounds to 1, so the BF16 logit
    is exactly 1 while the FP32 one keeps 1 + 2^-9."""
    s = np.zeros((1, 7))
    s[0, 0] = 1.0
    Ws = [np.array([[1.0 + 2.0 ** -9, 0, 0, 0, 0, 0, 0]]), np.zeros((1, 1)), np.zeros((1, 1)),
          np.ones((1, 1))]
    bs = [np.zeros(1), np.zeros(1), np.zeros(1), np.zeros(1)]
    assert orc.resnet_forward(s, Ws, bs, "bf16")[0, 0] == 1.0
    assert orc.resnet_forward(s, Ws, bs, "fp32")[0, 0] == 1.0 + 2.0 ** -9


def width_two_network():
    """The hand-computed width-two network above (one block, three outputs)."""
    s = np.zeros((1, 7))
    s[0, 0] = 1.0
    W_in = np.zeros((2, 7))
    W_in[0, 0], W_in[1, 0] = 2.0, -1.0
    Ws = [W_in, np.array([[1.0, 1.0], [0.0, -1.0]]), np.array([[0.5, 0.0], [1.0, -1.0]]),
          np.array([[1.0, 0.0], [0.0, 1.0], [1.0, -1.0]])]
    bs = [np.array([0.0, 3.0]), np.array([0.0, 1.0]), np.array([-1.0, 0.0]),
          np.array([0.0, 0.0, 10.0])]
    return s, Ws, bs


# magnitudes of the width-two network, by hand: input layer |W_in| |s| + |b_in| =
# [2, 0 + ... ] = [2, 1 + 3] = [2, 4]; block layer 1: [[1, 1], [0, 1]] [2, 4] + [0, 1] =
# [6, 5]; block layer 2 plus the residual: [[0.5, 0], [1, 1]] [6, 5] + [1, 0] + [2, 4] =
# [6, 15]; output: [[1, 0], [0, 1], [1, 1]] [6, 15] + [0, 0, 10] = [6, 15, 31]
WIDTH_TWO_MAGS = [[[2.0, 4.0]], [[6.0, 5.0]], [[6.0, 15.0]], [[6.0, 15.0, 31.0]]]


def test_magnitudes_hand_computed_width_two():
    """Every magnitude of the width-two network, exactly (the logits [3, 6, 7] are
    strictly inside them, so an over-estimate is caught as well as an under-estimate)."""
    s, Ws, bs = width_two_network()
    mags = orc.resnet_abs_forward(s, Ws, bs)
    assert [m.tolist() for m in mags] == WIDTH_TWO_MAGS


def test_magnitudes_bound_every_logit():
    rng = np.random.default_rng(5)
    Ws, bs = _model(32, 6, 7, rng)
    s = rng.random((100, 7))
    z = orc.resnet_forward(s, Ws, bs, "fp32")
    mags = orc.resnet_abs_forward(s, Ws, bs)
    assert len(mags) == 2 + 2 * 6
    assert (np.abs(z) <= mags[-1] * (1 + 1e-12)).all()
