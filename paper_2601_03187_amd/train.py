"""Weights for the tuple predictor (tooling, outside the classify path).

Training follows the recipe of Sec. 6.2 in reduced form: each packet's label is the
tuple of its highest-priority matching rule, obtained here from the library's own exact
classification; cross-entropy loss, Adam, batch 8192, learning rate 1e-3. The paper's
class-balance loop (alpha oversampling, beta accuracy target, 1000-epoch rounds) is
not run: the answers the library returns never depend on the weights, only the number
of tuples probed does.

Also: the static per-layer activation scales for FP8 (amax of each hidden layer's
output over a calibration batch, divided by 448) and random / degenerate weights used
by the weight-independence tests.
"""
from __future__ import annotations

import numpy as np

from . import tang as T

FEATURES = 104


def feature_bits_torch(hdr: np.ndarray, device="cpu"):
    """(n, 104) float32 tensor of header bits, MSB first: SIP, DIP, SP, DP, PROTO."""
    import torch
    words = [(hdr["sip"].astype(np.int64), 32), (hdr["dip"].astype(np.int64), 32),
             (hdr["sp"].astype(np.int64), 16), (hdr["dp"].astype(np.int64), 16),
             (hdr["proto"].astype(np.int64), 8)]
    cols = []
    for v, width in words:
        t = torch.as_tensor(v, device=device)
        shifts = torch.arange(width - 1, -1, -1, device=device)
        cols.append(((t[:, None] >> shifts[None, :]) & 1).to(torch.float32))
    return torch.cat(cols, dim=1)


def tuple_labels(rs: int, rules: np.ndarray, rule_ids: np.ndarray) -> np.ndarray:
    """Tuple index of each answered rule id (-1 for no match)."""
    ids = rules["id"].astype(np.int64)
    tup = np.array([T.tang_ruleset_rule_tuple(rs, int(i)) for i in ids], dtype=np.int64)
    order = np.argsort(ids)
    sid = ids[order]
    out = np.full(len(rule_ids), -1, dtype=np.int64)
    ok = rule_ids != T.TANG_NO_MATCH
    pos = np.searchsorted(sid, rule_ids[ok].astype(np.int64))
    out[ok] = tup[order[pos]]
    return out


def train_mlp(X, y, n_out: int, hidden: int, steps: int = 400, batch: int = 8192, lr: float = 1e-3,
              seed: int = 0, device="cpu"):
    """Plain 104 -> H -> H -> C MLP with ReLU. Returns ([W1, W2, W3], [b1, b2, b3]) as
    float32 numpy arrays ([out][in] layout)."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    torch.manual_seed(seed)
    net = torch.nn.Sequential(torch.nn.Linear(FEATURES, hidden), torch.nn.ReLU(),
                              torch.nn.Linear(hidden, hidden), torch.nn.ReLU(),
                              torch.nn.Linear(hidden, n_out)).to(device)
    opt = torch.optim.Adam(net.parameters(), lr=lr)
    X = X.to(device)
    y = torch.as_tensor(y, device=device)
    n = X.shape[0]
    for _ in range(steps):
        idx = torch.randint(0, n, (min(batch, n),), generator=g).to(device)
        loss = torch.nn.functional.cross_entropy(net(X[idx]), y[idx])
        opt.zero_grad()
        loss.backward()
        opt.step()
    Ws = [net[i].weight.detach().float().cpu().numpy().copy() for i in (0, 2, 4)]
    bs = [net[i].bias.detach().float().cpu().numpy().copy() for i in (0, 2, 4)]
    return Ws, bs


def accuracy(Ws, bs, X, y) -> float:
    import torch
    with torch.no_grad():
        h = X
        for l, (W, b) in enumerate(zip(Ws, bs)):
            h = h @ torch.as_tensor(W, device=X.device).T + torch.as_tensor(b, device=X.device)
            if l < len(Ws) - 1:
                h = torch.relu(h)
        return float((h.argmax(1).cpu().numpy() == y).mean())


def act_scales(Ws, bs, X) -> list:
    """[1, amax(h1)/448, amax(h2)/448] over the calibration batch X (FP32 forward)."""
    import torch
    out = [1.0]
    with torch.no_grad():
        h = X
        for l in range(len(Ws) - 1):
            h = torch.relu(h @ torch.as_tensor(Ws[l], device=X.device).T
                           + torch.as_tensor(bs[l], device=X.device))
            amax = float(h.abs().max())
            out.append(amax / 448.0 if amax > 0 else 1.0)
    return out


def random_weights(n_out: int, hidden: int, seed: int, scale: float = 1.0):
    rng = np.random.default_rng(seed)
    dims = [FEATURES, hidden, hidden, n_out]
    Ws = [(rng.standard_normal((dims[i + 1], dims[i])) * scale / np.sqrt(dims[i])).astype(np.float32)
          for i in range(3)]
    bs = [(rng.standard_normal(dims[i + 1]) * 0.1).astype(np.float32) for i in range(3)]
    return Ws, bs


def constant_winner_weights(n_out: int, hidden: int, winner: int):
    """All-zero weights with an output bias that makes `winner` the argmax everywhere."""
    dims = [FEATURES, hidden, hidden, n_out]
    Ws = [np.zeros((dims[i + 1], dims[i]), dtype=np.float32) for i in range(3)]
    bs = [np.zeros(dims[i + 1], dtype=np.float32) for i in range(3)]
    bs[2][winner] = 1.0
    return Ws, bs


def fit(rs: int, rules: np.ndarray, hdr: np.ndarray, hidden: int, steps: int = 400, seed: int = 0,
        device="cpu", rule_ids: np.ndarray | None = None):
    """Label `hdr` through the library (exact answers), train, and return
    (Ws, bs, act_scales, train_accuracy)."""
    import torch
    if rule_ids is None:
        rule_ids = T.tang_classify_host(rs, hdr)
    y = tuple_labels(rs, rules, rule_ids)
    keep = y >= 0
    X = feature_bits_torch(hdr[keep], device=device)
    yk = y[keep]
    C = T.tang_ruleset_num_tuples(rs)
    Ws, bs = train_mlp(X, yk, C, hidden, steps=steps, seed=seed, device=device)
    acc = accuracy(Ws, bs, X, yk)
    sc = act_scales(Ws, bs, X[: min(len(yk), 65536)])
    del torch
    return Ws, bs, sc, acc
