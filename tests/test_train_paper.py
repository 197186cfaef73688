"""The paper's training loop (Sec. 6.2) on the CPU: alpha oversampling and the beta rounds.
Labels come from the oracle here (the library labels through the GPU)."""
import numpy as np

from oracle import oracle as orc
from paper_2601_03187_amd import synth, train
from paper_2601_03187_amd import tang as T


def test_oversample_raises_small_classes_to_alpha_only():
    rng = np.random.default_rng(0)
    y = np.array([0] * 50 + [1] * 3 + [3] * 7)  # class 2 empty
    idx = train.oversample(y, 10, rng)
    counts = np.bincount(y[idx], minlength=4)
    assert counts.tolist() == [50, 10, 0, 10]
    assert set(np.arange(len(y))) <= set(idx.tolist())  # every sample at least once


def _tiny():
    rules = synth.make_rules(200, seed=7)
    hdr = synth.make_packets(rules, 3000, seed=8, frac_in=1.0)
    rs = T.tang_ruleset_create(T.TANG_HOST_ONLY, rules)
    return rules, hdr, rs, orc.classify(rules, hdr)


def test_beta_loop_multiplies_alpha_until_target():
    rules, hdr, rs, ids = _tiny()
    try:
        # an unreachable target: every round runs, alpha x 10 each time
        _, _, info = train.train_paper(rs, rules, hdr, hidden=32, alpha=5, beta=1.01, rounds=3,
                                       epochs=1, batch=512, rule_ids=ids)
        assert [r["alpha"] for r in info["rounds"]] == [5, 50, 500]
        assert not info["converged"]
        assert info["rounds"][2]["samples"] >= info["rounds"][0]["samples"]
        # a target met at once: one round, converged
        Ws, bs, info = train.train_paper(rs, rules, hdr, hidden=32, alpha=5, beta=0.0, rounds=3,
                                         epochs=1, batch=512, rule_ids=ids)
        assert len(info["rounds"]) == 1 and info["converged"]
        C = T.tang_ruleset_num_tuples(rs)
        assert [w.shape for w in Ws] == [(32, 104), (32, 32), (C, 32)]
    finally:
        T.tang_ruleset_destroy(rs)


def test_residual_network_export_matches_oracle_forward():
    """The trained residual network's exported weights, run through the oracle's forward
    pass (FP32), give the module's own logits: the export order and Eq. 1 agree."""
    import torch
    rules, hdr, rs, ids = _tiny()
    try:
        Ws, bs, info = train.train_paper(rs, rules, hdr, arch="resnet", hidden=16, n_blocks=2,
                                         alpha=5, beta=0.0, rounds=1, epochs=1, batch=512,
                                         rule_ids=ids)
        assert len(Ws) == 2 + 2 * 2 and Ws[0].shape == (16, 7)
        S = orc.segments(hdr[:50])
        want = orc.resnet_forward(S, Ws, bs, "fp32")
        net = train._resnet_module(T.tang_ruleset_num_tuples(rs), 16, 2)
        layers = [net.inp] + [l for blk in net.blocks for l in blk] + [net.out]
        with torch.no_grad():
            for l, W, b in zip(layers, Ws, bs):
                l.weight.copy_(torch.as_tensor(W))
                l.bias.copy_(torch.as_tensor(b))
            got = net(train.segments_torch(hdr[:50])).double().numpy()
        assert np.allclose(got, want, rtol=1e-4, atol=1e-5)
    finally:
        T.tang_ruleset_destroy(rs)
