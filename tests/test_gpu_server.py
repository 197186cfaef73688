"""Serving loop: continuous batching over several rulesets. Each request's answers are
the same whether it runs alone or mixed with others (integer results: tolerance 0), and
equal the oracle's."""
import time

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2601_03187_amd import synth, train
from paper_2601_03187_amd import tang as T
from tests._gpu import torch_cuda

pytestmark = pytest.mark.gpu


def _rulesets():
    out = []
    for k, (n, prec) in enumerate([(1000, "bf16"), (5000, "fp8"), (20_000, None)]):
        rules = synth.make_rules(n, seed=600 + k)
        rs = T.tang_ruleset_create(0, rules)
        if prec:
            C = T.tang_ruleset_num_tuples(rs)
            Ws, bs = train.random_weights(C, 256, seed=k)
            T.tang_model_load(rs, Ws, bs, prec, act_scales=[1.0, 0.05, 0.05] if prec == "fp8" else None)
        out.append((rules, rs))
    return out


@pytest.mark.parametrize("graphs,limit", [(1, 0), (0, 0), (1, 20_000)])
def test_alone_equals_mix(graphs, limit):
    torch_cuda()
    sets = _rulesets()
    srv = T.tang_server_create(0, n_streams=3, max_batch=16384, use_graphs=graphs,
                               max_inflight_packets=limit)
    try:
        tags = [T.tang_server_add_ruleset(srv, rs) for _, rs in sets]
        rng = np.random.default_rng(graphs * 10 + (limit > 0))
        reqs = []
        for q in range(90):
            tag = int(rng.integers(0, 3))
            n = int(np.floor(np.exp(rng.uniform(np.log(32), np.log(16384)))))
            hdr = synth.make_packets(sets[tag][0], n, seed=1000 + q, frac_in=0.8)
            out = np.full(n, 0xDEADBEEF, dtype=np.uint32)
            reqs.append((tag, hdr, out, T.tang_server_submit(srv, tags[tag], hdr, out)))
            if q % 7 == 0:
                time.sleep(0.001)  # some arrive while others are on the GPU
        for tag, hdr, out, r in reqs:
            T.tang_server_wait(r, 60_000_000)
            s, a, d = T.tang_server_req_times(r)
            assert 0 < s <= a <= d
            alone = T.tang_classify_host(sets[tag][1], hdr)
            assert np.array_equal(out, alone)
            assert np.array_equal(out, orc.classify(sets[tag][0], hdr))
            T.tang_server_req_free(r)
        # an update bumps the ruleset version: graphs are captured again
        ins = synth.make_rules(50, seed=999, ordering="literal")
        ins["id"] += 1_000_000
        ins["priority"] = 0
        T.tang_insert(sets[0][1], ins)
        allr = np.concatenate([sets[0][0], ins])
        hdr = synth.make_packets(allr, 3000, seed=5, frac_in=0.9)
        out = np.zeros(3000, dtype=np.uint32)
        r = T.tang_server_submit(srv, tags[0], hdr, out)
        T.tang_server_wait(r, 60_000_000)
        assert np.array_equal(out, orc.classify(allr, hdr))
        T.tang_server_req_free(r)
        # limits: a request that can never be admitted, and an empty one
        big = np.zeros(20_000, dtype=synth.HDR_DTYPE)
        with pytest.raises(T.TangError) as e:
            T.tang_server_submit(srv, tags[0], big, np.zeros(20_000, dtype=np.uint32))
        assert e.value.name == "EBUSY"
        r = T.tang_server_submit(srv, tags[0], np.zeros(0, dtype=synth.HDR_DTYPE), np.zeros(0, dtype=np.uint32))
        assert T.tang_server_poll(r)
        T.tang_server_req_free(r)
        with pytest.raises(T.TangError) as e:
            T.tang_server_submit(srv, 7, hdr, out)
        assert e.value.name == "EINVAL"
    finally:
        T.tang_server_destroy(srv)
        for _, rs in sets:
            T.tang_ruleset_destroy(rs)


def test_rulesets_added_while_serving():
    """Rulesets added while batches of earlier ones are in flight (the server's ruleset
    table grows from 1 to 17 entries meanwhile): every request's answers equal the
    oracle's."""
    torch_cuda()
    sets = []
    for k in range(17):
        rules = synth.make_rules(400 + 50 * k, seed=700 + k)
        rs = T.tang_ruleset_create(0, rules)
        if k % 2:
            C = T.tang_ruleset_num_tuples(rs)
            Ws, bs = train.random_weights(C, 128, seed=k)
            T.tang_model_load(rs, Ws, bs, "bf16")
        sets.append((rules, rs))
    srv = T.tang_server_create(0, n_streams=2, max_batch=4096, use_graphs=1)
    try:
        tags, reqs = [], []
        for k, (rules, rs) in enumerate(sets):
            tags.append(T.tang_server_add_ruleset(srv, rs))
            for q in range(4):
                tag = tags[(k + q) % len(tags)]
                hdr = synth.make_packets(sets[tag][0], 1000 + 700 * q, seed=2000 + 10 * k + q, frac_in=0.8)
                out = np.full(len(hdr), 0xDEADBEEF, dtype=np.uint32)
                reqs.append((tag, hdr, out, T.tang_server_submit(srv, tag, hdr, out)))
        assert tags == list(range(17))
        for tag, hdr, out, r in reqs:
            T.tang_server_wait(r, 60_000_000)
            assert np.array_equal(out, orc.classify(sets[tag][0], hdr)), tag
            T.tang_server_req_free(r)
    finally:
        T.tang_server_destroy(srv)
        for _, rs in sets:
            T.tang_ruleset_destroy(rs)


def test_alone_equals_mix_at_serving_sizes():
    """The serving workload's shape: resident rulesets of 10,000, 100,000 and 524,288
    rules with BF16 predictors, requests of log-uniform size 32..65,536 with a uniform
    ruleset tag, submitted in bursts while earlier ones run, 4 streams, graphs: every
    answer of every request equals the same headers classified alone, and a seeded
    sample of each request equals the oracle's."""
    torch_cuda()
    cfg = synth.CONFIGS["c5_serving"]
    sets = []
    for k, n_rules in enumerate(cfg["sizes"]):
        rules = synth.make_rules(n_rules, seed=cfg["seed"] + k, ordering="specificity")
        rs = T.tang_ruleset_create(0, rules)
        C = T.tang_ruleset_num_tuples(rs)
        Ws, bs = train.random_weights(C, cfg["hidden"], seed=50 + k)
        T.tang_model_load(rs, Ws, bs, "bf16")
        sets.append((rules, rs))
    srv = T.tang_server_create(0, n_streams=4, max_batch=65536, use_graphs=1)
    try:
        tags = [T.tang_server_add_ruleset(srv, rs) for _, rs in sets]
        _, sizes, tg = synth.make_requests(120, len(sets), seed=77, rate_per_s=1.0)
        reqs = []
        for q in range(len(sizes)):
            hdr = synth.make_packets(sets[tg[q]][0], int(sizes[q]), seed=3000 + q, frac_in=cfg["frac_in"])
            out = np.full(len(hdr), 0xDEADBEEF, dtype=np.uint32)
            reqs.append((int(tg[q]), hdr, out, T.tang_server_submit(srv, tags[tg[q]], hdr, out)))
            if q % 10 == 9:
                time.sleep(0.002)
        rng = np.random.default_rng(78)
        for tag, hdr, out, r in reqs:
            T.tang_server_wait(r, 120_000_000)
            assert np.array_equal(out, T.tang_classify_host(sets[tag][1], hdr)), tag
            k = rng.choice(len(hdr), size=min(len(hdr), 300), replace=False)
            assert np.array_equal(out[k], orc.classify(sets[tag][0], hdr[k])), tag
            T.tang_server_req_free(r)
    finally:
        T.tang_server_destroy(srv)
        for _, rs in sets:
            T.tang_ruleset_destroy(rs)


def test_prepared_graphs_serve_every_size_class():
    """tang_server_prepare records the graph of every size class on every slot; requests
    of every class afterwards (one header below, at and above each power of two, so the
    live count differs from the class), and again after a new model bumps the ruleset's
    version, all equal the oracle's answers. A bad tag is refused."""
    torch_cuda()
    rules = synth.make_rules(3000, seed=810)
    rs = T.tang_ruleset_create(0, rules)
    C = T.tang_ruleset_num_tuples(rs)
    Ws, bs = train.random_weights(C, 256, seed=11)
    T.tang_model_load(rs, Ws, bs, "bf16")
    srv = T.tang_server_create(0, n_streams=2, max_batch=8192, use_graphs=1)
    try:
        tag = T.tang_server_add_ruleset(srv, rs)
        T.tang_server_prepare(srv, tag)
        T.tang_server_prepare(srv, tag)   # already prepared: returns at once
        with pytest.raises(T.TangError) as e:
            T.tang_server_prepare(srv, tag + 1)
        assert e.value.name == "EINVAL"
        sizes = sorted({max(1, min(8192, (1 << p) + d)) for p in range(5, 14) for d in (-1, 0, 1)})
        for round_ in range(2):
            reqs = []
            for q, n in enumerate(sizes):
                hdr = synth.make_packets(rules, n, seed=4000 + 100 * round_ + q, frac_in=0.8)
                out = np.full(n, 0xDEADBEEF, dtype=np.uint32)
                reqs.append((hdr, out, T.tang_server_submit(srv, tag, hdr, out)))
            for hdr, out, r in reqs:
                T.tang_server_wait(r, 60_000_000)
                assert np.array_equal(out, orc.classify(rules, hdr)), (round_, len(hdr))
                T.tang_server_req_free(r)
            Wf, bf = train.random_weights(C, 256, seed=12)
            T.tang_model_load(rs, Wf, bf, "bf16", topk=2)
    finally:
        T.tang_server_destroy(srv)
        T.tang_ruleset_destroy(rs)


def test_residual_model_batches_beside_graph_batches():
    """A ruleset with the residual predictor (its batches run eagerly: the staging kernels,
    then the classification, on the slot's stream) served beside a BF16 ruleset (graph
    replays), requests of 1 to 8,192 headers alternating between the two: every answer
    equals the oracle's."""
    from tests.test_gpu_resnet import _random_model

    torch_cuda()
    sets = []
    for k in range(2):
        rules = synth.make_rules(2000, seed=820 + k)
        rs = T.tang_ruleset_create(0, rules)
        C = T.tang_ruleset_num_tuples(rs)
        if k == 0:
            Ws, bs = _random_model(C, 2, np.random.default_rng(821))
            T.tang_model_load_resnet(rs, Ws, bs, "bf16", topk=2)
        else:
            Ws, bs = train.random_weights(C, 256, seed=822)
            T.tang_model_load(rs, Ws, bs, "bf16")
        sets.append((rules, rs))
    srv = T.tang_server_create(0, n_streams=3, max_batch=8192, use_graphs=1)
    try:
        tags = [T.tang_server_add_ruleset(srv, rs) for _, rs in sets]
        for t in tags:
            T.tang_server_prepare(srv, t)
        reqs = []
        for q, n in enumerate([1, 33, 100, 4095, 4096, 5000, 8192, 7, 1000, 8191]):
            tag = q % 2
            hdr = synth.make_packets(sets[tag][0], n, seed=5000 + q, frac_in=0.8)
            out = np.full(n, 0xDEADBEEF, dtype=np.uint32)
            reqs.append((tag, hdr, out, T.tang_server_submit(srv, tags[tag], hdr, out)))
        for tag, hdr, out, r in reqs:
            T.tang_server_wait(r, 60_000_000)
            assert np.array_equal(out, orc.classify(sets[tag][0], hdr)), (tag, len(hdr))
            T.tang_server_req_free(r)
    finally:
        T.tang_server_destroy(srv)
        for _, rs in sets:
            T.tang_ruleset_destroy(rs)


def test_copy_engine_batches_beside_staged_ones():
    """Batches of more than 65,536 headers move through the copy engines, issued by the
    slot's own thread; smaller ones through the staging kernels. A burst that merges into
    batches of both kinds (a 200,000-header request, 65,536-header requests that merge up
    to 262,144, small ones), before and after a new model: every answer equals the
    oracle's."""
    torch_cuda()
    rules = synth.make_rules(3000, seed=830)
    rs = T.tang_ruleset_create(0, rules)
    C = T.tang_ruleset_num_tuples(rs)
    Ws, bs = train.random_weights(C, 256, seed=831)
    T.tang_model_load(rs, Ws, bs, "bf16")
    srv = T.tang_server_create(0, n_streams=2, max_batch=262144, use_graphs=1)
    try:
        tag = T.tang_server_add_ruleset(srv, rs)
        T.tang_server_prepare(srv, tag)
        sizes = [200_000, 65_536, 65_536, 65_536, 65_536, 33, 131_072, 70_000, 1, 65_536, 4_096]
        for round_ in range(2):
            reqs = []
            for q, n in enumerate(sizes):
                hdr = synth.make_packets(rules, n, seed=6000 + 100 * round_ + q, frac_in=0.8)
                out = np.full(n, 0xDEADBEEF, dtype=np.uint32)
                reqs.append((hdr, out, T.tang_server_submit(srv, tag, hdr, out)))
            for hdr, out, r in reqs:
                T.tang_server_wait(r, 60_000_000)
                assert np.array_equal(out, orc.classify(rules, hdr)), (round_, len(hdr))
                T.tang_server_req_free(r)
            Wf, bf = train.random_weights(C, 256, seed=832)
            T.tang_model_load(rs, Wf, bf, "bf16", topk=2)
    finally:
        T.tang_server_destroy(srv)
        T.tang_ruleset_destroy(rs)
