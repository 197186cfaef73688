"""Reader for tests/golden/tab_rules.txt (the worked example of Table 1, Sec. 4.1)."""
import os

import numpy as np

from paper_2601_03187_amd.synth import RULE_DTYPE, HDR_DTYPE

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _pattern(p):
    """A 3-bit pattern like '00*' -> (value of the top 3 bits of a 32-bit word, length)."""
    length = len(p.rstrip("*"))
    bits = p.replace("*", "0")
    return int(bits, 2) << 29, length


def make_rule(name, prio, x, y):
    r = np.zeros(1, dtype=RULE_DTYPE)[0]
    r["sip"], r["sip_len"] = _pattern(x)
    r["dip"], r["dip_len"] = _pattern(y)
    r["sp_lo"], r["sp_hi"], r["dp_lo"], r["dp_hi"] = 0, 65535, 0, 65535
    r["proto"], r["proto_mask"] = 0, 0
    r["priority"] = prio
    r["id"] = int(name[1:])
    return r


def load_tab_rules():
    rules, tuples, grid, inserts, changes, conflict = [], [], {}, [], [], {}
    with open(os.path.join(GOLDEN, "tab_rules.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            t = line.split()
            if t[0] == "rule":
                rules.append((t[1], int(t[2]), t[3], t[4], t[5]))
            elif t[0] == "tuple":
                tuples.append((t[1], int(t[2]), int(t[3])))
            elif t[0] == "grid":
                y = int(t[1])
                for x, cell in enumerate(t[2:]):
                    grid[(x, y)] = None if cell == "--" else cell
            elif t[0] == "insert":
                inserts.append((t[1], int(t[2]), t[3], t[4], t[5]))
            elif t[0] == "change":
                changes.append((int(t[1]), int(t[2]), t[3]))
            elif t[0] == "conflict":
                conflict[t[1]] = [] if t[2] == "-" else t[2:]
    arr = np.array([make_rule(n, p, x, y) for (n, p, x, y, _) in rules], dtype=RULE_DTYPE)
    return dict(rules=rules, array=arr, tuples=tuples, grid=grid, inserts=inserts,
                changes=changes, conflict=conflict)


def grid_packets(rng, reps=4):
    """Every (X, Y) point `reps` times with random low bits, ports and protocol."""
    pts = [(x, y) for y in range(8) for x in range(8)] * reps
    h = np.zeros(len(pts), dtype=HDR_DTYPE)
    low = (1 << 29) - 1
    for i, (x, y) in enumerate(pts):
        h[i]["sip"] = (x << 29) | int(rng.integers(0, low + 1))
        h[i]["dip"] = (y << 29) | int(rng.integers(0, low + 1))
        h[i]["sp"] = int(rng.integers(0, 65536))
        h[i]["dp"] = int(rng.integers(0, 65536))
        h[i]["proto"] = int(rng.integers(0, 256))
    return pts, h
