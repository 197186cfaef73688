"""The library's internal device memory through a caller's allocator (tang_set_allocator),
here torch's caching allocator: every block the library takes is returned, and the
answers are the oracle's, through a build, a model load, updates that grow the record
array and the slot table, and the residual model's workspace."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2601_03187_amd import synth, train
from paper_2601_03187_amd import tang as T
from tests._gpu import classify_dev, torch_cuda

pytestmark = pytest.mark.gpu


def test_internal_memory_through_callers_allocator():
    torch_cuda()
    live, calls = {}, {"alloc": 0, "free": 0}
    talloc, tfree = T.torch_allocator()

    def alloc(nbytes, dev):
        p = talloc(nbytes, dev)
        if p:
            calls["alloc"] += 1
            live[p] = nbytes
        return p

    def free(p, dev):
        calls["free"] += 1
        assert live.pop(p, None) is not None, hex(p)
        tfree(p, dev)

    T.tang_set_allocator(alloc, free)
    try:
        rules = synth.make_rules(5_000, seed=81)
        rs = T.tang_ruleset_create(0, rules)
        try:
            assert calls["alloc"] >= 5 and all(p % 256 == 0 for p in live)
            C = T.tang_ruleset_num_tuples(rs)
            T.tang_model_load(rs, *train.random_weights(C, 256, seed=3), "bf16", topk=2)
            hdr = synth.make_packets(rules, 50_000, seed=82, frac_in=0.8)
            assert np.array_equal(classify_dev(rs, hdr), orc.classify(rules, hdr))
            # enough fresh rules to grow the record array and rebuild the slot table
            ins = synth.make_rules(40_000, seed=83)
            ins["id"] += 1_000_000
            before = calls["alloc"]
            T.tang_insert(rs, ins)
            T.tang_delete(rs, rules["id"][::3])
            assert calls["alloc"] > before
            every = np.concatenate([rules, ins])
            lm = ~np.isin(every["id"], rules["id"][::3])
            pk = synth.make_packets(every[lm], 50_000, seed=84, frac_in=0.8)
            assert np.array_equal(classify_dev(rs, pk), orc.classify(every, pk, live=lm))
            rng = np.random.default_rng(5)
            Wr = [rng.normal(0, 2.0, (512, 7))] + [rng.normal(0, 1 / np.sqrt(512), (512, 512)) for _ in range(2)]
            Wr.append(rng.normal(0, 1 / np.sqrt(512), (C, 512)))
            br = [rng.normal(0, 0.05, w.shape[0]) for w in Wr]
            T.tang_model_load_resnet(rs, [w.astype(np.float32) for w in Wr],
                                     [b.astype(np.float32) for b in br], "bf16")
            assert max(live.values()) >= 3 * 65536 * 512 * 2  # the workspace came from torch
            assert np.array_equal(classify_dev(rs, pk), orc.classify(every, pk, live=lm))
        finally:
            T.tang_ruleset_destroy(rs)
        assert not live, f"{len(live)} blocks not returned"
        assert calls["free"] == calls["alloc"]
    finally:
        T.tang_set_allocator()


def test_serving_loop_slots_through_callers_allocator():
    """The serving loop's device slots come from the caller's allocator too and go back
    on destroy; its answers are the oracle's."""
    torch_cuda()
    live = {}
    talloc, tfree = T.torch_allocator()

    def alloc(nbytes, dev):
        p = talloc(nbytes, dev)
        if p:
            live[p] = nbytes
        return p

    def free(p, dev):
        assert live.pop(p, None) is not None, hex(p)
        tfree(p, dev)

    T.tang_set_allocator(alloc, free)
    try:
        rules = synth.make_rules(3000, seed=85)
        rs = T.tang_ruleset_create(0, rules)
        srv = None
        try:
            T.tang_model_load(rs, *train.random_weights(T.tang_ruleset_num_tuples(rs), 128, seed=4), "bf16")
            n_before = len(live)
            srv = T.tang_server_create(0, n_streams=2, max_batch=4096, use_graphs=1)
            tag = T.tang_server_add_ruleset(srv, rs)
            assert len(live) > n_before  # the slots
            reqs = []
            for q in range(12):
                hdr = synth.make_packets(rules, 100 + 300 * q, seed=86 + q, frac_in=0.8)
                out = np.full(len(hdr), 0xDEADBEEF, dtype=np.uint32)
                reqs.append((hdr, out, T.tang_server_submit(srv, tag, hdr, out)))
            for hdr, out, r in reqs:
                T.tang_server_wait(r, 60_000_000)
                assert np.array_equal(out, orc.classify(rules, hdr))
                T.tang_server_req_free(r)
        finally:
            if srv is not None:
                T.tang_server_destroy(srv)
            T.tang_ruleset_destroy(rs)
        assert not live, f"{len(live)} blocks not returned"
    finally:
        T.tang_set_allocator()


def test_block_freed_on_a_busy_side_stream_is_not_written_early():
    """torch's caching allocator recycles a block as soon as it is freed in its stream's
    order, while work queued on that stream may still write it. Blocks freed on a busy
    side stream, then taken by a ruleset build on that stream: the library waits for the
    queued writes before filling its tables, so the answers are the oracle's."""
    torch = torch_cuda()
    talloc, tfree = T.torch_allocator()
    T.tang_set_allocator(talloc, tfree)
    side = torch.cuda.Stream()
    rs = None
    try:
        rules = synth.make_rules(4000, seed=87)
        hdr = synth.make_packets(rules, 20_000, seed=88, frac_in=0.8)
        with torch.cuda.stream(side):
            bufs = [torch.empty(1 << k, dtype=torch.uint8, device="cuda") for k in range(12, 25)]
            a = torch.ones(4096, 4096, device="cuda")
            c = torch.empty_like(a)
            for _ in range(30):               # tens of ms of queued work on the side stream
                torch.mm(a, a, out=c)
            for buf in bufs:
                buf.fill_(0xA5)               # runs after the products, into the freed blocks
            del bufs, buf, a, c
            rs = T.tang_ruleset_create(0, rules)
            C = T.tang_ruleset_num_tuples(rs)
            T.tang_model_load(rs, *train.random_weights(C, 128, seed=5), "bf16", topk=1)
        torch.cuda.synchronize()
        assert np.array_equal(classify_dev(rs, hdr), orc.classify(rules, hdr))
    finally:
        if rs is not None:
            T.tang_ruleset_destroy(rs)
        T.tang_set_allocator()


def test_failed_update_flush_leaves_the_ruleset_refusing_device_calls():
    """An insert whose device flush cannot allocate (the caller's allocator returns NULL
    while the record array grows) fails, and since the host side already holds the batch,
    the ruleset then refuses every device call (EDEVICE) instead of answering from tables
    that disagree with it. Its export still gives the intended live rules, and a ruleset
    rebuilt from them answers like the oracle."""
    torch_cuda()
    talloc, tfree = T.torch_allocator()
    state = {"fail": False}

    def alloc(nbytes, dev):
        return 0 if state["fail"] else talloc(nbytes, dev)

    T.tang_set_allocator(alloc, tfree)
    rs = rs2 = None
    try:
        rules = synth.make_rules(3000, seed=89)
        rs = T.tang_ruleset_create(0, rules)
        hdr = synth.make_packets(rules, 5000, seed=90, frac_in=0.8)
        assert np.array_equal(classify_dev(rs, hdr), orc.classify(rules, hdr))
        ins = synth.make_rules(80_000, seed=91)   # more than the record array's spare room
        ins["id"] += 1_000_000
        state["fail"] = True
        with pytest.raises(T.TangError) as e:
            T.tang_insert(rs, ins)
        assert e.value.name == "EDEVICE"
        state["fail"] = False
        for call in (lambda: classify_dev(rs, hdr), lambda: T.tang_delete(rs, rules["id"][:1]),
                     lambda: T.tang_insert(rs, ins[:1]),
                     lambda: T.tang_model_load(rs, *train.random_weights(
                         T.tang_ruleset_num_tuples(rs), 128, seed=6), "bf16")):
            with pytest.raises(T.TangError) as e:
                call()
            assert e.value.name == "EDEVICE"
        every = np.concatenate([rules, ins])
        exp = T.tang_ruleset_export(rs)
        assert np.array_equal(np.sort(exp["id"]), np.sort(every["id"]))
        rs2 = T.tang_ruleset_create(0, exp)
        pk = synth.make_packets(every, 20_000, seed=92, frac_in=0.8)
        assert np.array_equal(classify_dev(rs2, pk), orc.classify(every, pk))
    finally:
        for r in (rs, rs2):
            if r is not None:
                T.tang_ruleset_destroy(r)
        T.tang_set_allocator()
