"""CPU oracle for the batched packet-classification path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU-baseline
leg may import this module; the library and its binding never do. It shares no code
with the GPU path (the only common import is the seeded input generator, which holds
none of the method's arithmetic).

Contents, each written from the passage it cites:

* ``classify``            -- linear scan (C, ``tang_oracle.c``): highest-priority match
                             (Sec. 2.1), lower priority number wins (Table 1 / Sec. 4.2),
                             ties to the lower id.
* ``classify_definition`` -- the same definition as a literal argmin in pure Python, for
                             tiny inputs only.
* ``feature_bits``        -- the 104 header bits the model reads, MSB first over
                             SIP, DIP, SP, DP, PROTO.
* ``bf16_round`` / ``e4m3_round`` -- round-to-nearest-even onto the value sets of the
                             bfloat16 and OCP FP8 E4M3 formats, built by enumerating
                             each format's representable values from its definition.
* ``mlp_forward``         -- the plain MLP of Sec. 6.1 without residual blocks
                             (FC -> ReLU -> FC -> ReLU -> FC), in float64, with the
                             BF16 / FP8 quantisation steps emulated on the inputs of
                             each layer (FP8 weight scales: ``fp8_weight_scale``,
                             ``fp8_hidden_weight_scale``); ``topk`` picks predicted
                             tuples (argmax of Sec. 6.1, ties to the lower index).
* ``segments`` / ``resnet_forward`` -- the paper's own model input and network
                             (Sec. 6.2 input format, Sec. 6.1 with residual blocks,
                             Eq. 1, sizes of Sec. 7.1): seven 16-bit header chunks as
                             floats, FC -> ReLU, residual blocks, FC; float64 with the
                             BF16 rounding steps emulated.
* ``tuples_first_appearance`` / ``rule_tuples`` -- tuple space (Sec. 4.3): rules
                             grouped by their (SIP length, DIP length) signature,
                             numbered by first appearance in priority order (Table 1).
* ``insert_tuple``        -- restricted insertion (Sec. 5.2.1).
* ``conflict_masks``      -- brute force over rule pairs: for rule m, the tuples that
                             hold a higher-priority rule whose box intersects m's box.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tang_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
NO_MATCH = 0xFFFFFFFF
_lib = None


def build_oracle(force: bool = False) -> str:
    """Compile tang_oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fPIC", "-shared", "-pthread", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build_oracle()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_classify.restype = ctypes.c_int
        lib.oracle_classify.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int]
        _lib = lib
    return _lib


def default_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def classify(rules: np.ndarray, pkts: np.ndarray, live: np.ndarray | None = None,
             threads: int | None = None, want_scanned: bool = False):
    """Linear-scan answers (uint32 rule ids, 0xFFFFFFFF = no match)."""
    lib = _load()
    rules = np.ascontiguousarray(rules)
    pkts = np.ascontiguousarray(pkts)
    assert rules.dtype.itemsize == 28 and pkts.dtype.itemsize == 16
    out = np.empty(len(pkts), dtype=np.uint32)
    scanned = np.empty(len(pkts), dtype=np.uint64) if want_scanned else None
    lv = None
    if live is not None:
        lv = np.ascontiguousarray(live.astype(np.uint8))
    rc = lib.oracle_classify(rules.ctypes.data if len(rules) else None, len(rules),
                             lv.ctypes.data if lv is not None else None,
                             pkts.ctypes.data if len(pkts) else None, len(pkts),
                             out.ctypes.data if len(pkts) else None,
                             scanned.ctypes.data if scanned is not None and len(pkts) else None,
                             int(threads or default_threads()))
    if rc != 0:
        raise MemoryError("oracle_classify failed")
    return (out, scanned) if want_scanned else out


# ---------------------------------------------------------------------------------------
# The definition written out literally (tiny inputs only).

def prefix_mask(length: int) -> int:
    """Top `length` bits of a 32-bit word set; length 0 -> 0 (Sec. 4.3 truncation)."""
    length = int(length)
    return 0 if length == 0 else ((1 << 32) - (1 << (32 - length)))


def rule_matches(r, p) -> bool:
    """Sec. 2.1: IP prefixes, inclusive port ranges, exact-or-wildcard protocol."""
    ms, md = prefix_mask(r["sip_len"]), prefix_mask(r["dip_len"])
    return ((int(p["sip"]) & ms) == (int(r["sip"]) & ms)
            and (int(p["dip"]) & md) == (int(r["dip"]) & md)
            and int(r["sp_lo"]) <= int(p["sp"]) <= int(r["sp_hi"])
            and int(r["dp_lo"]) <= int(p["dp"]) <= int(r["dp_hi"])
            and (int(r["proto_mask"]) == 0 or int(p["proto"]) == int(r["proto"])))


def classify_definition(rules, pkts, live=None) -> np.ndarray:
    """argmin over matching live rules of (priority, id); NO_MATCH if none."""
    out = np.empty(len(pkts), dtype=np.uint32)
    for k, p in enumerate(pkts):
        best = None
        for i, r in enumerate(rules):
            if live is not None and not live[i]:
                continue
            if rule_matches(r, p):
                key = (int(r["priority"]), int(r["id"]))
                if best is None or key < best:
                    best = key
        out[k] = NO_MATCH if best is None else best[1]
    return out


# ---------------------------------------------------------------------------------------
# Model input: 104 header bits, MSB first, SIP(32) DIP(32) SP(16) DP(16) PROTO(8).

FIELDS = (("sip", 32), ("dip", 32), ("sp", 16), ("dp", 16), ("proto", 8))
N_FEATURES = 104


def feature_bits(pkts: np.ndarray) -> np.ndarray:
    cols = []
    for name, width in FIELDS:
        v = pkts[name].astype(np.uint64)
        for b in range(width - 1, -1, -1):
            cols.append(((v >> np.uint64(b)) & np.uint64(1)).astype(np.float64))
    return np.stack(cols, axis=1) if len(pkts) else np.zeros((0, N_FEATURES))


# ---------------------------------------------------------------------------------------
# Number formats, from their definitions.

def _bf16_values() -> np.ndarray:
    """All finite non-negative bfloat16 values: 1 sign, 8 exponent (bias 127), 7 fraction
    bits; exponent field 0 encodes subnormals f * 2^-133, 255 encodes inf/NaN."""
    e = np.arange(0, 255, dtype=np.float64)[:, None]
    f = np.arange(0, 128, dtype=np.float64)[None, :]
    normal = (1.0 + f / 128.0) * np.power(2.0, e - 127.0)
    sub = f / 128.0 * 2.0 ** -126
    vals = np.where(e == 0, sub, normal)
    return vals.reshape(-1)  # ascending in (e, f), i.e. by bit pattern


def _e4m3_values() -> np.ndarray:
    """All finite non-negative OCP FP8 E4M3 values: 4 exponent bits (bias 7), 3 fraction
    bits, no infinities; only S.1111.111 is NaN, so the largest value is 1.75 * 2^8 = 448.
    Exponent field 0 encodes subnormals f/8 * 2^-6."""
    vals = []
    for code in range(0, 0x7F):          # 0x7F is NaN
        e, f = code >> 3, code & 7
        vals.append(f / 8.0 * 2.0 ** -6 if e == 0 else (1.0 + f / 8.0) * 2.0 ** (e - 7))
    return np.array(vals, dtype=np.float64)


def _round_to_set(x: np.ndarray, vals: np.ndarray, saturate: bool) -> np.ndarray:
    """Nearest value of the ascending non-negative set `vals` (mirrored for negatives);
    an exact tie goes to the value whose code (index = bit pattern) is even."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    if saturate:
        a = np.minimum(a, vals[-1])
    hi = np.minimum(np.searchsorted(vals, a, side="left"), len(vals) - 1)
    lo = np.maximum(hi - 1, 0)
    dlo = a - vals[lo]
    dhi = vals[hi] - a
    take_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    r = np.where(take_hi, vals[hi], vals[lo])
    return np.copysign(r, x)


_BF16 = None
_E4M3 = None


def bf16_round(x) -> np.ndarray:
    global _BF16
    if _BF16 is None:
        _BF16 = _bf16_values()
    return _round_to_set(x, _BF16, saturate=False)


def e4m3_round(x) -> np.ndarray:
    """Saturating: magnitudes beyond 448 become 448 (the format has no infinity)."""
    global _E4M3
    if _E4M3 is None:
        _E4M3 = _e4m3_values()
    return _round_to_set(x, _E4M3, saturate=True)


E4M3_MAX = 448.0


# ---------------------------------------------------------------------------------------
# The MLP (Sec. 6.1, without residual blocks): layers l = 1..L, z_l = W_l a_{l-1} + b_l,
# h_l = ReLU(z_l) for hidden layers, logits = z_L. W_l is [out][in] (PyTorch Linear).

def fp8_weight_scale(W: np.ndarray) -> float:
    """Per-layer weight scale: amax(|W|) / 448 (1 for an all-zero layer), as fp32. The
    output layer uses it as is."""
    amax = float(np.max(np.abs(W))) if W.size else 0.0
    return float(np.float32(amax / E4M3_MAX)) if amax > 0 else 1.0


def fp8_hidden_weight_scale(W: np.ndarray, s_a: float, s_next: float) -> float:
    """Weight scale of a hidden layer whose input scale is s_a and whose output feeds a
    layer of input scale s_next: the amax scale s raised by a factor in [1, 2) so that the
    requantisation factor s_w s_a / s_next is a power of two 2^e, the least one not below
    s s_a / s_next; s_w = 2^e s_next / s_a, as fp32. (The layer's output then enters the
    next layer as E4M3(2^e (product sum + b / (s_a s_w))), a scaling without rounding.)"""
    s = fp8_weight_scale(W)
    k = float(s) * float(s_a) / float(s_next)
    mant, ex = math.frexp(k)          # k = mant 2^ex, mant in [0.5, 1)
    e = ex - 1 if mant == 0.5 else ex
    return float(np.float32(math.ldexp(float(s_next) / float(s_a), e)))


def mlp_forward(x: np.ndarray, Ws, bs, precision: str = "fp32", act_scales=None) -> np.ndarray:
    """Logits in float64. precision: fp32 (no rounding), bf16 (weights and layer inputs
    rounded to bfloat16), fp8 (layer inputs scaled by the given per-layer activation scale
    and weights by their layer's weight scale -- ``fp8_hidden_weight_scale`` for the
    hidden layers, amax/448 for the output layer -- both rounded to E4M3 with saturation;
    the product sum is multiplied back by s_a * s_w). Biases stay unrounded."""
    a = np.asarray(x, dtype=np.float64)
    L = len(Ws)
    for l in range(L):
        W = np.asarray(Ws[l], dtype=np.float64)
        b = np.asarray(bs[l], dtype=np.float64)
        if precision == "fp32":
            z = a @ W.T + b
        elif precision == "bf16":
            z = bf16_round(a) @ bf16_round(W).T + b
        elif precision == "fp8":
            # activation scales are fp32 values (the library's interface type)
            s_a = 1.0 if l == 0 else float(np.float32(act_scales[l]))
            s_w = (fp8_hidden_weight_scale(W, s_a, float(np.float32(act_scales[l + 1])))
                   if l < L - 1 else fp8_weight_scale(W))
            inv_a = float(np.float32(1.0 / s_a))
            inv_w = float(np.float32(1.0 / s_w))
            qa = e4m3_round(a * inv_a)
            qw = e4m3_round(W * inv_w)
            deq = float(np.float32(np.float32(s_a) * np.float32(s_w)))
            z = (qa @ qw.T) * deq + b
        else:
            raise ValueError(precision)
        a = np.maximum(z, 0.0) if l < L - 1 else z
    return a


def mlp_abs_forward(x: np.ndarray, Ws, bs) -> list:
    """Per-layer magnitudes m_l = |W_l| m_{l-1} + |b_l| with m_0 = |x| (float64). By the
    triangle inequality m_l bounds |z_l| and |ReLU(z_l)| entrywise, so it scales the
    accumulated rounding error of every layer; with non-negative weights, biases and
    inputs it equals the forward pass itself."""
    a = np.abs(np.asarray(x, dtype=np.float64))
    mags = []
    for l, (W, b) in enumerate(zip(Ws, bs)):
        m = a @ np.abs(np.asarray(W, np.float64)).T + np.abs(np.asarray(b, np.float64))
        mags.append(m)
        a = m
    return mags


def segments(pkts: np.ndarray) -> np.ndarray:
    """The model input of Sec. 6.2: the header cut into 16-bit chunks -- SIP high, SIP low,
    DIP high, DIP low, SP, DP, PROTO -- each turned into a float. The scale is unstated;
    read here as the chunk value divided by 65535, so every input lies in [0, 1]."""
    sip = pkts["sip"].astype(np.int64)
    dip = pkts["dip"].astype(np.int64)
    cols = [sip >> 16, sip & 0xFFFF, dip >> 16, dip & 0xFFFF,
            pkts["sp"].astype(np.int64), pkts["dp"].astype(np.int64), pkts["proto"].astype(np.int64)]
    return np.stack(cols, axis=1).astype(np.float64) / 65535.0


def resnet_forward(s: np.ndarray, Ws, bs, precision: str = "bf16") -> np.ndarray:
    """Logits (float64) of the network of Sec. 6.1 with residual blocks: an input FC layer
    with ReLU, then blocks B(x) = relu(relu(x w1 + b1) w2 + b2 + x) (Eq. 1, its unbalanced
    parentheses read as the usual residual block with the ReLU after the sum), then an
    output FC layer without activation. Ws = [W_in, W_11, W_12, ..., W_k1, W_k2, W_out]
    in nn.Linear layout [out][in], bs likewise. The input layer (seven inputs) is computed
    unrounded; with precision "bf16" every later layer's weights and inputs are rounded to
    bfloat16 (the residual term x is the rounded block input), biases stay unrounded."""
    if precision == "fp32":
        rnd = lambda a: a  # noqa: E731
    elif precision == "bf16":
        rnd = bf16_round
    else:
        raise ValueError(precision)
    f64 = lambda a: np.asarray(a, dtype=np.float64)  # noqa: E731
    a = np.maximum(f64(s) @ f64(Ws[0]).T + f64(bs[0]), 0.0)
    n_blocks = (len(Ws) - 2) // 2
    for k in range(n_blocks):
        W1, b1, W2, b2 = Ws[1 + 2 * k], bs[1 + 2 * k], Ws[2 + 2 * k], bs[2 + 2 * k]
        x = rnd(a)
        h = np.maximum(x @ rnd(f64(W1)).T + f64(b1), 0.0)
        a = np.maximum(rnd(h) @ rnd(f64(W2)).T + f64(b2) + x, 0.0)
    return rnd(a) @ rnd(f64(Ws[-1])).T + f64(bs[-1])


def resnet_abs_forward(s: np.ndarray, Ws, bs) -> list:
    """Magnitudes after every layer, for error bounds: m = |W_in| |s| + |b_in|, then per
    block h = |w1| m + |b1| and m <- |w2| h + |b2| + m (the residual term enters with its
    own magnitude), then |W_out| m + |b_out|. Returned in that order (input layer, the
    two layers of each block, output layer)."""
    f64 = lambda a: np.abs(np.asarray(a, dtype=np.float64))  # noqa: E731
    a = f64(s) @ f64(Ws[0]).T + f64(bs[0])
    mags = [a]
    for k in range((len(Ws) - 2) // 2):
        h = a @ f64(Ws[1 + 2 * k]).T + f64(bs[1 + 2 * k])
        a = h @ f64(Ws[2 + 2 * k]).T + f64(bs[2 + 2 * k]) + a
        mags += [h, a]
    mags.append(a @ f64(Ws[-1]).T + f64(bs[-1]))
    return mags


def topk(logits: np.ndarray, k: int) -> np.ndarray:
    """Indices of the k largest logits per row, larger first, ties to the lower index."""
    idx = np.argsort(-logits, axis=1, kind="stable")
    return idx[:, :k]


def mlp_flops(dims, padded_dims=None) -> int:
    """2 * sum(in * out) over the layers (one multiply and one add per weight)."""
    d = padded_dims or dims
    return int(sum(2 * d[i] * d[i + 1] for i in range(len(d) - 1)))


# ---------------------------------------------------------------------------------------
# Tuple space (Sec. 4.3) and restricted insertion (Sec. 5.2.1).

def tuples_first_appearance(rules: np.ndarray, live=None) -> list:
    """Distinct (sip_len, dip_len) signatures in order of first appearance when the rules
    are visited by ascending (priority, id)."""
    idx = [i for i in range(len(rules)) if live is None or live[i]]
    idx.sort(key=lambda i: (int(rules[i]["priority"]), int(rules[i]["id"])))
    seen = []
    for i in idx:
        sig = (int(rules[i]["sip_len"]), int(rules[i]["dip_len"]))
        if sig not in seen:
            seen.append(sig)
    return seen


def rule_tuples(rules: np.ndarray) -> np.ndarray:
    tup = tuples_first_appearance(rules)
    pos = {s: i for i, s in enumerate(tup)}
    return np.array([pos[(int(r["sip_len"]), int(r["dip_len"]))] for r in rules], dtype=np.int64)


def insert_tuple(tuples: list, sip_len: int, dip_len: int) -> int:
    """Restricted insertion: the tuple with the identical signature if there is one;
    otherwise, among tuples whose every length is <= the rule's, the first one with the
    largest length sum. -1 if no tuple qualifies."""
    for i, (a, b) in enumerate(tuples):
        if a == sip_len and b == dip_len:
            return i
    best, best_sum = -1, -1
    for i, (a, b) in enumerate(tuples):
        if a <= sip_len and b <= dip_len and a + b > best_sum:
            best, best_sum = i, a + b
    return best


def _box(r):
    ms, md = prefix_mask(r["sip_len"]), prefix_mask(r["dip_len"])
    s0 = int(r["sip"]) & ms
    d0 = int(r["dip"]) & md
    proto = None if int(r["proto_mask"]) == 0 else int(r["proto"])
    return ((s0, s0 | (~ms & 0xFFFFFFFF)), (d0, d0 | (~md & 0xFFFFFFFF)),
            (int(r["sp_lo"]), int(r["sp_hi"])), (int(r["dp_lo"]), int(r["dp_hi"])), proto)


def boxes_intersect(r1, r2) -> bool:
    b1, b2 = _box(r1), _box(r2)
    for (lo1, hi1), (lo2, hi2) in zip(b1[:4], b2[:4]):
        if hi1 < lo2 or hi2 < lo1:
            return False
    return b1[4] is None or b2[4] is None or b1[4] == b2[4]


def conflict_masks(rules: np.ndarray, tuple_of: np.ndarray) -> np.ndarray:
    """mask[m] = OR of bit tuple_of[r] over rules r with (priority, id) below m's whose
    box intersects m's box (pairwise brute force; small rulesets only)."""
    n = len(rules)
    out = np.zeros(n, dtype=object)  # Python ints: any number of tuples
    keys = [(int(r["priority"]), int(r["id"])) for r in rules]
    for m in range(n):
        acc = 0
        for r in range(n):
            if keys[r] < keys[m] and boxes_intersect(rules[r], rules[m]):
                acc |= 1 << int(tuple_of[r])
        out[m] = acc
    return out
