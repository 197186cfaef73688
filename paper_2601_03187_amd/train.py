"""Weights for the tuple predictor (tooling, outside the classify path).

Labels follow Sec. 6.2: each packet's label is the tuple of its highest-priority
matching rule, obtained here from the library's own exact classification. ``fit`` trains
the plain predictor in reduced form (cross-entropy, Adam, batch 8192, learning rate 1e-3,
a fixed number of steps); ``train_paper`` runs the paper's whole loop: classes below a
threshold alpha are oversampled up to alpha, rounds of epochs with the learning rate
decayed by 0.1 every fifth of a round, and alpha multiplied by 10 after any round whose
accuracy stays below beta. The answers the library returns never depend on the weights,
only the number of tuples probed does.

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


def segments_torch(hdr: np.ndarray, device="cpu"):
    """(n, 7) float32 tensor of the residual predictor's input (Sec. 6.2): SIP high, SIP low,
    DIP high, DIP low, SP, DP, PROTO, each divided by 65535."""
    import torch
    sip = hdr["sip"].astype(np.int64)
    dip = hdr["dip"].astype(np.int64)
    cols = [sip >> 16, sip & 0xFFFF, dip >> 16, dip & 0xFFFF, hdr["sp"].astype(np.int64),
            hdr["dp"].astype(np.int64), hdr["proto"].astype(np.int64)]
    return torch.as_tensor(np.stack(cols, axis=1), device=device).to(torch.float32) / 65535.0


def _resnet_module(n_out: int, width: int, n_blocks: int):
    """Sec. 6.1 with residual blocks: FC(7 -> width) + ReLU, blocks
    relu(relu(x w1 + b1) w2 + b2 + x), FC(width -> C)."""
    import torch

    class Net(torch.nn.Module):
        def __init__(self):
            super().__init__()
            self.inp = torch.nn.Linear(7, width)
            self.blocks = torch.nn.ModuleList(
                [torch.nn.ModuleList([torch.nn.Linear(width, width), torch.nn.Linear(width, width)])
                 for _ in range(n_blocks)])
            self.out = torch.nn.Linear(width, n_out)

        def forward(self, x):
            x = torch.relu(self.inp(x))
            for l1, l2 in self.blocks:
                x = torch.relu(l2(torch.relu(l1(x))) + x)
            return self.out(x)

        def layers(self):
            return [self.inp] + [l for blk in self.blocks for l in blk] + [self.out]

        def export(self):
            return ([l.weight.detach().float().cpu().numpy().copy() for l in self.layers()],
                    [l.bias.detach().float().cpu().numpy().copy() for l in self.layers()])

    return Net()


def _mlp_module(n_out: int, hidden: int):
    import torch

    class Net(torch.nn.Sequential):
        def layers(self):
            return [self[i] for i in (0, 2, 4)]

        def export(self):
            return ([l.weight.detach().float().cpu().numpy().copy() for l in self.layers()],
                    [l.bias.detach().float().cpu().numpy().copy() for l in self.layers()])

    return Net(torch.nn.Linear(FEATURES, hidden), torch.nn.ReLU(), torch.nn.Linear(hidden, hidden),
               torch.nn.ReLU(), torch.nn.Linear(hidden, n_out))


def oversample(y: np.ndarray, alpha: int, rng: np.random.Generator) -> np.ndarray:
    """Indices of the training set: every sample once, plus, for each class with fewer
    than alpha samples, random repeats of its samples up to alpha (empty classes stay
    empty)."""
    idx = [np.arange(len(y))]
    classes, counts = np.unique(y, return_counts=True)
    for c, k in zip(classes, counts):
        if k < alpha:
            idx.append(rng.choice(np.flatnonzero(y == c), int(alpha - k), replace=True))
    return np.concatenate(idx)


def train_paper(rs: int, rules: np.ndarray, hdr: np.ndarray, *, arch: str = "mlp", hidden: int = 256,
                n_blocks: int = 6, alpha: int = 1000, beta: float = 0.95, rounds: int = 4,
                epochs: int = 5, batch: int = 8192, lr: float = 1e-3, seed: int = 0, device="cpu",
                rule_ids: np.ndarray | None = None, init=None, log=None):
    """The training loop of Sec. 6.2 (epochs per round reduced from the paper's 1000):
    labels from TSS lookups, alpha oversampling, cross-entropy with Adam, the learning rate
    multiplied by 0.1 after every fifth of a round's epochs, and after each round alpha x 10
    unless the accuracy on the (not oversampled) labelled set reaches beta. The model is
    kept across rounds (reading: the paper regenerates the set, not the model).
    arch "mlp": the plain 104-bit predictor; "resnet": the paper's residual network.
    init = (Ws, bs) starts from existing weights (the incremental training of Sec. 5.2.2).
    Returns (Ws, bs, info) with info = {"rounds": [{"alpha", "samples", "accuracy"}],
    "converged": bool}."""
    import torch
    if rule_ids is None:
        rule_ids = T.tang_classify_host(rs, hdr)
    y = tuple_labels(rs, rules, rule_ids)
    keep = y >= 0
    y = y[keep]
    C = T.tang_ruleset_num_tuples(rs)
    X = (feature_bits_torch if arch == "mlp" else segments_torch)(hdr[keep], device=device)
    torch.manual_seed(seed)
    net = (_mlp_module(C, hidden) if arch == "mlp" else _resnet_module(C, hidden, n_blocks)).to(device)
    if init is not None:
        with torch.no_grad():
            for layer, W, b in zip(net.layers(), init[0], init[1]):
                layer.weight.copy_(torch.as_tensor(W))
                layer.bias.copy_(torch.as_tensor(b))
    yt = torch.as_tensor(y, device=device)
    rng = np.random.default_rng(seed)
    info = {"rounds": [], "converged": False}
    for _ in range(rounds):
        idx = oversample(y, alpha, rng)
        opt = torch.optim.Adam(net.parameters(), lr=lr)
        sched = torch.optim.lr_scheduler.StepLR(opt, step_size=max(1, epochs // 5), gamma=0.1)
        for _ in range(epochs):
            perm = torch.as_tensor(rng.permutation(idx), device=device)
            for s in range(0, len(perm), batch):
                b = perm[s:s + batch]
                loss = torch.nn.functional.cross_entropy(net(X[b]), yt[b])
                opt.zero_grad()
                loss.backward()
                opt.step()
            sched.step()
        with torch.no_grad():
            pred = torch.cat([net(X[s:s + 65536]).argmax(1) for s in range(0, len(y), 65536)])
            acc = float((pred == yt).float().mean())
        info["rounds"].append({"alpha": int(alpha), "samples": int(len(idx)), "accuracy": acc})
        if log:
            log(f"[train] round {len(info['rounds'])}: alpha {alpha}, {len(idx)} samples, accuracy {acc:.4f}")
        if acc >= beta:
            info["converged"] = True
            break
        alpha *= 10
    Ws, bs = net.export()
    return Ws, bs, info


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
