"""The deferred update (Sec. 5.2.2) end to end on the GPU: windows of drifting updates
(deletes, and inserts with a SIP prefix length the tuple set lacks, which restricted
insertion puts in coarser tuples), the policy's decision from each window's lookup cost,
then the update it asks for -- incremental training (the current model fine-tuned on
fresh labels and reloaded) or a full rebuild (a new tuple space from the exported live
rules and a model trained from scratch) -- and after every window and every update the
answers equal the oracle's scan of the live rules.

The policy watches throughput; here its input is the reciprocal of the search's memory
accesses per header (filter words, slots and records, counted by the kernel), which is
what the throughput follows and, unlike a timing, repeats exactly run to run. Models are
trained on the CPU, so the whole sequence of decisions is fixed by the seeds."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2601_03187_amd import synth, train
from paper_2601_03187_amd import tang as T
from paper_2601_03187_amd.deferred import DeferredUpdate
from tests._gpu import classify_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _train(rs, live, seed, init=None, epochs=3):
    h = synth.make_packets(live, 1 << 16, seed=seed, frac_in=0.8)
    Ws, bs, _ = train.train_paper(rs, live, h, hidden=128, alpha=200, beta=0.0, rounds=1,
                                  epochs=epochs, seed=seed, device="cpu", init=init)
    T.tang_model_load(rs, Ws, bs, "bf16", topk=1)
    return Ws, bs


def _check(rs, live, seed):
    hdr = synth.make_packets(live, 60_000, seed=seed, frac_in=0.8)
    got, st = classify_dev(rs, hdr, stats=True)
    assert np.array_equal(got, orc.classify(live, hdr)), seed
    n = st["packets"]
    return n / (st["filter_checks"] + st["slots"] + st["records"])


def test_drift_windows_deferred_update_exact():
    torch_cuda()
    rules0 = synth.make_rules(16_384, seed=808, ordering="specificity")
    ups = synth.make_update_stream(rules0, 6, 800, seed=809, prio_range=len(rules0), sip_lengths=(4,))
    rs = T.tang_ruleset_create(0, rules0)
    pol = DeferredUpdate(tau=0.05, theta=1_200)
    actions = []
    try:
        model = _train(rs, rules0, 810, epochs=4)
        pol.observe(_check(rs, rules0, 811), T.tang_ruleset_coarse_rules(rs))
        for w, (ins, dels) in enumerate(ups, start=1):
            T.tang_delete(rs, dels)
            T.tang_insert(rs, ins)
            live = T.tang_ruleset_export(rs)
            print(f"window {w}: {len(live)} live rules, coarse {T.tang_ruleset_coarse_rules(rs)}", flush=True)
            th = _check(rs, live, 820 + w)
            act = pol.observe(th, T.tang_ruleset_coarse_rules(rs))
            actions.append(act)
            if act == "incremental":
                model = _train(rs, live, 830 + w, init=model, epochs=2)
            elif act == "full":
                T.tang_ruleset_destroy(rs)
                rs = None
                rs = T.tang_ruleset_create(0, live)
                assert T.tang_ruleset_coarse_rules(rs) == 0
                model = _train(rs, live, 840 + w, epochs=4)
            if act:
                pol.deployed(act)
                _check(rs, live, 850 + w)  # the updated model / tuple space, same rules
        assert "incremental" in actions and "full" in actions, actions
    finally:
        if rs is not None:
            T.tang_ruleset_destroy(rs)
