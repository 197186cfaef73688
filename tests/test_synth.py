"""Seeded input generator: determinism and the distributions the workloads name."""
import numpy as np

from paper_2601_03187_amd import synth


def test_same_seed_same_bytes():
    a = synth.make_rules(5000, seed=3, ordering="specificity", mix=0.25)
    b = synth.make_rules(5000, seed=3, ordering="specificity", mix=0.25)
    assert a.tobytes() == b.tobytes()
    pa = synth.make_packets(a, 10000, seed=4, frac_in=0.8, zipf_s=1.0)
    pb = synth.make_packets(b, 10000, seed=4, frac_in=0.8, zipf_s=1.0)
    assert pa.tobytes() == pb.tobytes()
    assert synth.make_rules(5000, seed=5).tobytes() != a.tobytes()


def test_prefix_length_histogram():
    r = synth.make_rules(200_000, seed=1, ordering="literal")
    for f in ("sip_len", "dip_len"):
        for L, p in zip(synth.IP_LENS, synth.IP_LEN_P):
            assert abs((r[f] == L).mean() - p) < 0.01
    # values are normalised to their prefix
    for f, lf in (("sip", "sip_len"), ("dip", "dip_len")):
        L = r[lf].astype(np.uint64)
        low = np.where(L == 0, np.uint64(0xFFFFFFFF), (np.uint64(1) << (np.uint64(32) - L)) - np.uint64(1))
        assert ((r[f].astype(np.uint64) & low) == 0).all()


def test_port_and_protocol_mix():
    r = synth.make_rules(200_000, seed=2, ordering="literal")
    wild = (r["sp_lo"] == 0) & (r["sp_hi"] == 65535)
    exact = r["sp_lo"] == r["sp_hi"]
    assert abs(wild.mean() - 0.60) < 0.01
    assert abs(exact.mean() - 0.25) < 0.01
    assert (r["sp_lo"] <= r["sp_hi"]).all() and (r["dp_lo"] <= r["dp_hi"]).all()
    assert set(np.unique(r["proto_mask"]).tolist()) == {0, 255}
    assert abs((r["proto_mask"] == 0).mean() - 0.25) < 0.01
    assert set(np.unique(r["proto"][r["proto_mask"] != 0]).tolist()) == {1, 6, 17}


def test_mix_shifts_lengths_to_wildcards():
    plain = synth.make_rules(100_000, seed=7, ordering="literal")
    mixed = synth.make_rules(100_000, seed=7, ordering="literal", mix=0.25)
    assert (mixed["sip_len"] == 0).mean() > (plain["sip_len"] == 0).mean() + 0.08


def test_specificity_order_is_nonincreasing_in_length_sum():
    r = synth.make_rules(20_000, seed=8, ordering="specificity")
    s = r["sip_len"].astype(int) + r["dip_len"].astype(int)
    assert (np.diff(s) <= 0).all()
    assert (r["priority"] == np.arange(len(r))).all() and (r["id"] == r["priority"]).all()


def test_packets_inside_and_zipf_skew():
    r = synth.make_rules(10_000, seed=9)
    p, src = synth.make_packets(r, 200_000, seed=10, frac_in=0.8, zipf_s=1.0, return_src=True)
    assert abs((src >= 0).mean() - 0.8) < 0.01
    counts = np.bincount(src[src >= 0], minlength=len(r))
    top = np.sort(counts)[::-1]
    # Zipf(1) over 10k items: the most popular rule takes ~1/H(10^4) ~ 10% of draws
    assert 0.07 < top[0] / counts.sum() < 0.14
    # headers lie inside their source rule's port ranges
    ins = src >= 0
    rr = r[src[ins]]
    assert ((p["sp"][ins] >= rr["sp_lo"]) & (p["sp"][ins] <= rr["sp_hi"])).all()


def test_update_stream_and_requests():
    r = synth.make_rules(1000, seed=11)
    ups = synth.make_update_stream(r, rounds=3, per_round=10, seed=12)
    assert len(ups) == 3
    ids = set(r["id"].tolist())
    for ins, dels in ups:
        assert set(dels.tolist()) <= ids
        ids -= set(dels.tolist())
        assert not (set(ins["id"].tolist()) & ids)
        ids |= set(ins["id"].tolist())
    t, sizes, tags = synth.make_requests(1000, 3, seed=13, rate_per_s=1000.0)
    assert (np.diff(t) > 0).all() and sizes.min() >= 32 and sizes.max() <= 65536
    assert set(np.unique(tags).tolist()) == {0, 1, 2}


def test_wide_generator_lengths_and_tuples():
    """wide=True: IP lengths uniform over the 12 WIDE_IP_LENS values per field, so a large
    ruleset covers all 144 (SIP, DIP) signatures; values stay normalised."""
    r = synth.make_rules(100_000, seed=9, wide=True)
    for f in ("sip_len", "dip_len"):
        vals, counts = np.unique(r[f], return_counts=True)
        assert vals.tolist() == sorted(synth.WIDE_IP_LENS.tolist())
        assert np.abs(counts / len(r) - 1 / 12).max() < 0.01
    sig = r["sip_len"].astype(np.int64) * 64 + r["dip_len"]
    assert len(np.unique(sig)) == 144
    L = r["sip_len"].astype(np.uint64)
    low = np.where(L == 0, np.uint64(0xFFFFFFFF), (np.uint64(1) << (np.uint64(32) - L)) - np.uint64(1))
    assert ((r["sip"].astype(np.uint64) & low) == 0).all()
