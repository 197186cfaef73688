"""Seeded synthetic inputs: 5-field rulesets, packet traces, update streams, request streams.

This module only draws inputs. It holds none of the classification arithmetic (no
matching, no tuple construction, no hashing), so both the GPU path and the CPU oracle
can be fed from it without sharing any of the method's code.

The paper measures on ClassBench-ng ACL/FW/IPC rulesets and on 1M-packet synthetic
traces whose packets fall inside randomly chosen rules (Sec. 7.1). Those files are not available here; the
generator below stands in for them with the field shapes of the problem statement
(Sec. 2.1: prefixes for the IPs, ranges for the ports, exact-or-wildcard protocol):

* IP prefix lengths, independently for SIP and DIP: {32: 40%, 24: 20%, 16: 15%,
  8: 10%, 0: 15%}; the value is uniform and masked to its length.
* Ports, independently for SP and DP: 60% wildcard [0, 65535], 25% exact [v, v],
  15% random range [min(a, b), max(a, b)].
* Protocol: uniform over {TCP=6, UDP=17, ICMP=1, *}.
* "Wildcard-heavy overlap mix" (optional fraction of rules): IP lengths {16: 25%,
  8: 25%, 0: 50%} and 90% port wildcards (the other 10% split exact:range = 25:15).
* Ordering: "literal" keeps generation order; "specificity" stable-sorts by
  descending sip_len + dip_len, then by port class (exact < range < wildcard, summed
  over SP and DP), then exact protocol before '*', before indices are assigned.
  Priority = id = final index (lower number = higher priority).
* Packets: a fraction is drawn inside a rule (each field uniform inside the rule's
  box; a wildcard protocol draws 0..255); the rest are uniform random 104-bit headers.
  Rule popularity is uniform or Zipf(s) over a seeded random permutation of the rules.

Every generator takes an explicit seed and uses numpy's PCG64, so the same seed gives
the same bytes on every machine.
"""
from __future__ import annotations

import numpy as np

# C layouts of tang_rule_t (28 B) and tang_header_t (16 B); see include/tang.h.
RULE_DTYPE = np.dtype([
    ("sip", "<u4"), ("dip", "<u4"), ("priority", "<u4"), ("id", "<u4"),
    ("sp_lo", "<u2"), ("sp_hi", "<u2"), ("dp_lo", "<u2"), ("dp_hi", "<u2"),
    ("sip_len", "u1"), ("dip_len", "u1"), ("proto", "u1"), ("proto_mask", "u1"),
])
HDR_DTYPE = np.dtype([
    ("sip", "<u4"), ("dip", "<u4"), ("sp", "<u2"), ("dp", "<u2"),
    ("proto", "u1"), ("pad", "u1", (3,)),
])
assert RULE_DTYPE.itemsize == 28 and HDR_DTYPE.itemsize == 16

NO_MATCH = 0xFFFFFFFF

IP_LENS = np.array([32, 24, 16, 8, 0], dtype=np.int64)
IP_LEN_P = np.array([0.40, 0.20, 0.15, 0.10, 0.15])
# a wide tuple space: 12 lengths per field, uniform -> 144 (SIP, DIP) signatures, in
# the range of the paper's rulesets (31-391 tuples)
WIDE_IP_LENS = np.array([32, 30, 28, 26, 24, 22, 20, 18, 16, 12, 8, 0], dtype=np.int64)
# every prefix length: the SIP length uniform over 0..32 and the DIP length within
# ALL_LEN_SPREAD of it (clipped to 0..32) -> 387 (SIP, DIP) signatures, near the paper's
# largest ruleset (391 tuples)
ALL_LEN_SPREAD = 6
MIX_IP_LENS = np.array([16, 8, 0], dtype=np.int64)
MIX_IP_LEN_P = np.array([0.25, 0.25, 0.50])
PORT_P = np.array([0.60, 0.25, 0.15])            # wildcard, exact, range
MIX_PORT_P = np.array([0.90, 0.0625, 0.0375])
PROTOS = np.array([6, 17, 1, -1], dtype=np.int64)  # -1 stands for '*'

PORT_WILD, PORT_EXACT, PORT_RANGE = 0, 1, 2


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _keep_bits(lens: np.ndarray) -> np.ndarray:
    """High `len` bits set, as uint64 (len in 0..32); used only to draw values."""
    lens = lens.astype(np.uint64)
    full = np.uint64(0xFFFFFFFF)
    out = np.where(lens == 0, np.uint64(0),
                   (full << (np.uint64(32) - np.maximum(lens, np.uint64(1)))) & full)
    return out.astype(np.uint64)


def _draw_ports(rng, n, probs):
    cls = rng.choice(3, size=n, p=probs)
    a = rng.integers(0, 65536, size=n)
    b = rng.integers(0, 65536, size=n)
    lo = np.where(cls == PORT_WILD, 0, np.where(cls == PORT_EXACT, a, np.minimum(a, b)))
    hi = np.where(cls == PORT_WILD, 65535, np.where(cls == PORT_EXACT, a, np.maximum(a, b)))
    return lo.astype(np.uint16), hi.astype(np.uint16), cls


def make_rules(n: int, seed: int, ordering: str = "specificity", mix: float = 0.0,
               wide: bool = False, all_lengths: bool = False) -> np.ndarray:
    """Draw `n` 5-field rules. Returns a RULE_DTYPE array with priority = id = index.
    wide: IP prefix lengths uniform over WIDE_IP_LENS (a tuple space of ~144 tuples).
    all_lengths: every prefix length 0..32 (see ALL_LEN_SPREAD; ~387 tuples)."""
    if ordering not in ("specificity", "literal"):
        raise ValueError(ordering)
    rng = _rng(seed)
    heavy = rng.random(n) < mix
    if all_lengths:
        sl = rng.integers(0, 33, size=n)
        dl = np.clip(sl + rng.integers(-ALL_LEN_SPREAD, ALL_LEN_SPREAD + 1, size=n), 0, 32)
    elif wide:
        sl = rng.choice(WIDE_IP_LENS, size=n)
        dl = rng.choice(WIDE_IP_LENS, size=n)
    else:
        sl = rng.choice(IP_LENS, size=n, p=IP_LEN_P)
        dl = rng.choice(IP_LENS, size=n, p=IP_LEN_P)
    if heavy.any():
        k = int(heavy.sum())
        sl[heavy] = rng.choice(MIX_IP_LENS, size=k, p=MIX_IP_LEN_P)
        dl[heavy] = rng.choice(MIX_IP_LENS, size=k, p=MIX_IP_LEN_P)
    sv = rng.integers(0, 1 << 32, size=n, dtype=np.uint64) & _keep_bits(sl)
    dv = rng.integers(0, 1 << 32, size=n, dtype=np.uint64) & _keep_bits(dl)
    splo, sphi, spc = _draw_ports(rng, n, PORT_P)
    dplo, dphi, dpc = _draw_ports(rng, n, PORT_P)
    if heavy.any():
        k = int(heavy.sum())
        a, b, c = _draw_ports(rng, k, MIX_PORT_P)
        splo[heavy], sphi[heavy], spc[heavy] = a, b, c
        a, b, c = _draw_ports(rng, k, MIX_PORT_P)
        dplo[heavy], dphi[heavy], dpc[heavy] = a, b, c
    pr = rng.choice(PROTOS, size=n)

    if ordering == "specificity":
        # port class rank: exact (0) < range (1) < wildcard (2)
        rank = np.array([2, 0, 1])
        port_score = rank[spc] + rank[dpc]
        proto_wild = (pr < 0).astype(np.int64)
        order = np.lexsort((proto_wild, port_score, -(sl + dl)))
    else:
        order = np.arange(n)

    r = np.zeros(n, dtype=RULE_DTYPE)
    r["sip"] = sv[order]
    r["dip"] = dv[order]
    r["sip_len"] = sl[order]
    r["dip_len"] = dl[order]
    r["sp_lo"], r["sp_hi"] = splo[order], sphi[order]
    r["dp_lo"], r["dp_hi"] = dplo[order], dphi[order]
    p = pr[order]
    r["proto"] = np.where(p < 0, 0, p)
    r["proto_mask"] = np.where(p < 0, 0, 0xFF)
    r["priority"] = np.arange(n, dtype=np.uint32)
    r["id"] = np.arange(n, dtype=np.uint32)
    return r


def _zipf_ranks(rng, n_items: int, count: int, s: float) -> np.ndarray:
    w = 1.0 / np.power(np.arange(1, n_items + 1, dtype=np.float64), s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(count)
    return np.minimum(np.searchsorted(cdf, u, side="right"), n_items - 1)


def sample_inside(rules: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    """One header drawn uniformly inside each given rule's box (protocol '*' -> 0..255)."""
    k = len(rules)
    h = np.zeros(k, dtype=HDR_DTYPE)
    for f, lf in (("sip", "sip_len"), ("dip", "dip_len")):
        keep = _keep_bits(rules[lf])
        rnd = rng.integers(0, 1 << 32, size=k, dtype=np.uint64)
        h[f] = ((rules[f].astype(np.uint64) & keep) | (rnd & ~keep & np.uint64(0xFFFFFFFF))).astype(np.uint32)
    for f in ("sp", "dp"):
        lo = rules[f + "_lo"].astype(np.int64)
        hi = rules[f + "_hi"].astype(np.int64)
        h[f] = rng.integers(lo, hi + 1).astype(np.uint16)
    anyp = rng.integers(0, 256, size=k)
    h["proto"] = np.where(rules["proto_mask"] != 0, rules["proto"], anyp).astype(np.uint8)
    return h


def random_headers(n: int, rng: np.random.Generator) -> np.ndarray:
    h = np.zeros(n, dtype=HDR_DTYPE)
    h["sip"] = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    h["dip"] = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    h["sp"] = rng.integers(0, 65536, size=n)
    h["dp"] = rng.integers(0, 65536, size=n)
    h["proto"] = rng.integers(0, 256, size=n)
    return h


def make_packets(rules: np.ndarray, n: int, seed: int, frac_in: float,
                 zipf_s: float | None = None, return_src: bool = False):
    """Draw `n` headers: a `frac_in` share inside rules (uniform or Zipf popularity over a
    seeded permutation of the rules), the rest uniform random. With return_src, also
    return the index of the rule each header was drawn from (-1 for random ones)."""
    rng = _rng(seed)
    inside = rng.random(n) < frac_in
    k = int(inside.sum())
    nr = len(rules)
    src = np.full(n, -1, dtype=np.int64)
    h = random_headers(n, rng)
    if k and nr:
        if zipf_s is None:
            idx = rng.integers(0, nr, size=k)
        else:
            perm = rng.permutation(nr)
            idx = perm[_zipf_ranks(rng, nr, k, zipf_s)]
        h[inside] = sample_inside(rules[idx], rng)
        src[inside] = idx
    return (h, src) if return_src else h


def make_update_stream(rules: np.ndarray, rounds: int, per_round: int, seed: int,
                       prio_range: int | None = None, sip_lengths=None):
    """Interleaved update rounds: each round is (inserts, delete_ids). Inserted rules come
    from the same field generator, priority uniform in [0, prio_range), fresh ids from
    max(id)+1 upward; deletes are uniform among the ids live at that point. With
    `sip_lengths`, the inserted rules' SIP prefix lengths are drawn uniformly from it
    instead (a drifting rule distribution) and their SIPs masked to those lengths."""
    rng = _rng(seed)
    live = list(int(i) for i in rules["id"])
    next_id = int(rules["id"].max()) + 1 if len(rules) else 0
    if prio_range is None:
        prio_range = max(1, len(rules))
    out = []
    for rd in range(rounds):
        ins = make_rules(per_round, seed=int(rng.integers(0, 2**62)), ordering="literal")
        if sip_lengths is not None:
            ln = rng.choice(np.asarray(sip_lengths), size=per_round).astype(np.uint8)
            mask = np.where(ln == 0, 0, (0xFFFFFFFF << (32 - ln.astype(np.uint64))) & 0xFFFFFFFF)
            ins["sip_len"] = ln
            ins["sip"] = (ins["sip"].astype(np.uint64) & mask).astype(np.uint32)
        ins["priority"] = rng.integers(0, prio_range, size=per_round).astype(np.uint32)
        ins["id"] = np.arange(next_id, next_id + per_round, dtype=np.uint32)
        next_id += per_round
        # deletes are drawn from rules live before this round's inserts
        pick = rng.choice(len(live), size=min(per_round, len(live)), replace=False)
        dels = np.array(sorted((live[i] for i in pick)), dtype=np.uint32)
        dset = set(int(x) for x in dels)
        live = [x for x in live if x not in dset] + [int(x) for x in ins["id"]]
        out.append((ins, dels))
    return out


def make_requests(n_requests: int, n_rulesets: int, seed: int, rate_per_s: float,
                  min_size: int = 32, max_size: int = 65536):
    """Poisson arrivals with log-uniform batch sizes floor(exp(U[ln min, ln max])) and a
    uniform ruleset tag. Returns (arrival_s, size, tag) arrays."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps)
    sizes = np.floor(np.exp(rng.uniform(np.log(min_size), np.log(max_size), size=n_requests)))
    sizes = np.clip(sizes.astype(np.int64), min_size, max_size)
    tags = rng.integers(0, n_rulesets, size=n_requests)
    return t, sizes, tags


# Named workloads: sizes and seeds of the five benchmark configurations.
CONFIGS = {
    "c1_1k": dict(n_rules=1024, n_pkts=10_000, frac_in=0.70, zipf=None, mix=0.0,
                  hidden=128, seed=101),
    "c2_64k": dict(n_rules=65_536, n_pkts=1_000_000, frac_in=0.80, zipf=None, mix=0.25,
                   hidden=256, seed=202),
    "c3_512k": dict(n_rules=524_288, n_pkts=16_777_216, frac_in=1.00, zipf=1.0, mix=0.0,
                    hidden=256, seed=303),
    "c4_512k_updates": dict(n_rules=524_288, n_pkts=1_000_000, frac_in=0.80, zipf=None,
                            mix=0.0, hidden=256, seed=404, rounds=100, per_round=100),
    "c5_serving": dict(sizes=(10_000, 100_000, 524_288), frac_in=0.80, hidden=256, seed=505),
    # a wide tuple space (144 tuples): 512k rules, 16M Zipf headers
    "c7_wide": dict(n_rules=524_288, n_pkts=16_777_216, frac_in=1.0, zipf=1.0, mix=0.0,
                    hidden=256, seed=707),
    # every prefix length 0..32 (387 tuples, the size of the paper's largest tuple
    # spaces): 512k rules, 16M Zipf headers
    "c8_all_lengths": dict(n_rules=524_288, n_pkts=16_777_216, frac_in=1.0, zipf=1.0,
                           mix=0.0, hidden=256, seed=808),
    # the paper's dynamic experiment (Sec. 7.4) scaled to one GPU: windows of deletes and
    # inserts with a SIP prefix length the tuple set does not have (a drifting
    # distribution; one new length keeps a rebuilt tuple space within 32 tuples)
    "c6_drift": dict(n_rules=65_536, windows=10, per_window=2_000, n_pkts=1_000_000,
                     frac_in=0.80, hidden=256, seed=606, sip_lengths=(4,)),
}
