#!/usr/bin/env python3
"""Throughput benchmark: Mpps classified at 512k rules on one MI355X.

Workload (one "step" = one tang_classify over the whole batch, headers already resident
in HBM): 524,288 synthetic 5-field rules in specificity order, 16,777,216 headers drawn
inside rules with Zipf(s=1) rule popularity, MLP 104 -> 256 -> 256 -> C trained on
labels from the library's exact answers. The headline line is the BF16 predictor; FP32
and FP8 are measured beside it, all with bit-exact rule ids (checked against the oracle
on a seeded sample). Also reported: per-step latency percentiles, per-kernel times with
the roofline of the dominant kernel, probes/records per header, and the oracle's CPU
throughput on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 20] [--warmup 5]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = {"k_mlp": "paper_2601_03187_amd/csrc/k_mlp.hip",
                  "k_classify": "paper_2601_03187_amd/csrc/k_classify.hip"}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_sha(rel: str) -> str:
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when the
    kernel source changed since the counters were taken."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_sha") != source_sha(KERNEL_SOURCES[kernel]):
        return None
    return t.get("traffic_bytes_per_launch")


def library_gather(dev, table_bytes: int) -> dict:
    """For scale: independent random 4-byte gathers through torch's indexing kernel over a
    table as large as the search's tables (so it sits where they sit: the Infinity Cache,
    not HBM), 2^26 indices, mean of 5 launches."""
    import torch
    g = torch.Generator(device=dev)
    g.manual_seed(5)
    words = table_bytes // 4
    tab = torch.randint(0, 1 << 30, (words,), dtype=torch.int32, device=dev, generator=g)
    n_idx = 1 << 26
    idx = torch.randint(0, words, (n_idx,), device=dev, generator=g)
    res = tab[idx]
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(5):
        res = tab[idx]
    b.record()
    torch.cuda.synchronize()
    rate = n_idx / (a.elapsed_time(b) / 5 * 1e-3)
    del tab, idx, res
    return {"table_bytes": int(words * 4), "indices": n_idx, "gathers_per_s": rate,
            "how": "torch advanced indexing, 4-byte elements"}


def search_alg_bytes(slots: float, records: float, matched: float) -> float:
    """Algorithmic bytes of the search per header: the 13-byte header, the 4-byte rule id,
    16 bytes per hash slot read, 32 per rule record compared, and 4 for the conflict mask
    of a matched rule."""
    return 13 + 4 + 16 * slots + 32 * records + 4 * matched


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precisions", default="bf16,fp32,fp8")
    ap.add_argument("--ordering", default="specificity", choices=["specificity", "literal"])
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--cpu-sample", type=int, default=200_000)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-literal", action="store_true")
    ap.add_argument("--skip-probe-all", action="store_true")
    ap.add_argument("--skip-hybrid", action="store_true",
                    help="skip the paper's CPU-GPU split (GPU predicts, host threads search)")
    ap.add_argument("--skip-stats", action="store_true",
                    help="skip the paper's training loop and its statistics (model accuracy, "
                         "classification accuracy of the paper's own search, memory accesses)")
    ap.add_argument("--skip-resnet", action="store_true",
                    help="skip the paper-size residual predictor (7 -> 512 -> 6 blocks -> C)")
    ap.add_argument("--skip-configs", action="store_true",
                    help="skip the 1k / 64k configurations and the 80%%-rule-sampled 512k run")
    ap.add_argument("--workload", default="c3", choices=["c3", "c4", "c5", "c6"],
                    help="c3: 512k rules / 16M headers (the headline line); c4: the update "
                         "stream on the 512k ruleset; c5: the serving loop over three rulesets; "
                         "c6: drifting updates with and without the deferred update")
    ap.add_argument("--rounds", type=int, default=100, help="c4: update rounds")
    ap.add_argument("--update-sample", type=int, default=1000,
                    help="c4: headers of each round's batch checked against the oracle's re-scan")
    ap.add_argument("--skip-updates", action="store_true", help="skip the c4 update stream")
    ap.add_argument("--skip-serving", action="store_true", help="skip the c5 serving loop")
    ap.add_argument("--skip-drift", action="store_true", help="skip the c6 drift experiment")
    ap.add_argument("--requests", type=int, default=2000, help="c5: requests per load level")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run a plain device copy of this many bytes (3 times), the "
                         "reference kernel that calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); classification "
              "shards by replicating the ruleset per GPU and splitting batches, so N GPUs give "
              "N x the one-GPU rate -- run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2601_03187_amd import synth, train
    from paper_2601_03187_amd import tang as T

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.workload == "c4":
        return print_updates(bench_updates(args))
    if args.workload == "c5":
        return print_serving(bench_serving(args))
    if args.workload == "c6":
        return print_drift(bench_drift(args))
    if args.copy_bytes:
        a = torch.empty(args.copy_bytes // 4, dtype=torch.int32, device=dev).fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log(f"[bench] copy calibration: 3 x {args.copy_bytes} bytes")
    cfg = synth.CONFIGS["c3_512k"]
    n = cfg["n_pkts"]
    t0 = time.time()
    rules = synth.make_rules(cfg["n_rules"], seed=cfg["seed"], ordering=args.ordering)
    hdr, src = synth.make_packets(rules, n, seed=cfg["seed"] + 1, frac_in=cfg["frac_in"],
                                  zipf_s=cfg["zipf"], return_src=True)
    log(f"[bench] generated {len(rules)} rules, {n} headers in {time.time() - t0:.1f}s")
    t0 = time.time()
    rs = T.tang_ruleset_create(0, rules)
    build_s = time.time() - t0
    C = T.tang_ruleset_num_tuples(rs)
    table_bytes = T.tang_ruleset_device_bytes(rs)  # before any model: the search's tables
    log(f"[bench] ruleset built in {build_s:.2f}s, {C} tuples, {table_bytes} device bytes")
    d_hdr = torch.from_numpy(hdr.view(np.uint8).reshape(-1)).to(dev)
    d_out = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    t0 = time.time()
    Ws, bs, sc, acc = train.fit(rs, rules, hdr[: 1 << 18], cfg["hidden"], steps=args.train_steps,
                                seed=1, device="cuda")
    log(f"[bench] predictor trained in {time.time() - t0:.1f}s, top-1 train accuracy {acc:.3f}")

    H = cfg["hidden"]
    flop_pkt = 2 * (104 * H + H * H + H * C)
    per = {}
    got_by_prec = {}
    for prec in args.precisions.split(","):
        T.tang_model_load(rs, Ws, bs, prec, topk=1, act_scales=sc if prec == "fp8" else None)
        st = T.tang_classify(rs, d_hdr, d_out, n, stream, want_stats=True)
        got_by_prec[prec] = d_out.cpu().numpy().view(np.uint32).copy()
        for _ in range(args.warmup):
            T.tang_classify(rs, d_hdr, d_out, n, stream)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        w0 = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            T.tang_classify(rs, d_hdr, d_out, n, stream)
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        step_ms = [a.elapsed_time(b) for a, b in ev]
        # the two stages on their own, same stream, HIP events around each launch
        ek = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(args.steps)]
        for a, b, c in ek:
            a.record(stream)
            T.tang_predict(rs, d_hdr, d_out, n, stream)
            b.record(stream)
            T.tang_search(rs, d_hdr, d_out, n, stream)
            c.record(stream)
        torch.cuda.synchronize()
        k1 = float(np.mean([a.elapsed_time(b) for a, b, _ in ek]))
        k23 = float(np.mean([b.elapsed_time(c) for _, b, c in ek]))
        assert np.array_equal(d_out.cpu().numpy().view(np.uint32), got_by_prec[prec])
        S = st["slots"] / n
        E = st["records"] / n
        F = st["filter_checks"] / n
        matched = 1.0 - st["no_match"] / n
        # algorithmic bytes of the search per header: header in, rule id out, the slots and
        # records the method reads, and a matched rule's conflict mask; the bucket-filter
        # blocks (8 bytes each) and the candidate word read back from the predictor are
        # this implementation's own traffic, reported beside it
        bytes_pkt = search_alg_bytes(S, E, matched)
        impl_pkt = 8 * F + 4
        per[prec] = dict(
            mpps=n * args.steps / wall / 1e6, ms_per_step=wall * 1e3 / args.steps,
            p50_ms=pct(step_ms, 50), p99_ms=pct(step_ms, 99),
            k_mlp_ms=k1, k_classify_ms=k23,
            mlp_tflops=flop_pkt * n / (k1 * 1e-3) / 1e12,
            mlp_frac=flop_pkt * n / (k1 * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
            search_gbs=bytes_pkt * n / (k23 * 1e-3) / 1e9,
            probes_per_pkt=st["probes"] / n, slots_per_pkt=S, records_per_pkt=E,
            top1_hit_rate=st["top1_hits"] / n, fallback_rate=st["fallbacks"] / n,
            filter_checks_per_pkt=F, wave_steps=st["wave_steps"] / n,
            wave_rounds=st["wave_rounds"] / n, search_bytes_per_pkt=bytes_pkt,
            search_overhead_bytes_per_pkt=impl_pkt, matched_rate=matched)
        # stage rooflines in Mpps: the predictor at its MFMA peak, the search at HBM peak
        # over its algorithmic bytes; serial = both back to back, overlap = the slower one
        k1_mpps = PEAK_TFLOPS[prec] * 1e12 / flop_pkt / 1e6
        k2_mpps = PEAK_HBM_GBS * 1e9 / bytes_pkt / 1e6
        serial = 1.0 / (1.0 / k1_mpps + 1.0 / k2_mpps)
        per[prec]["roofline_mpps"] = dict(k_mlp=k1_mpps, k_classify=k2_mpps, serial=serial,
                                          overlapped=min(k1_mpps, k2_mpps),
                                          frac_of_serial=per[prec]["mpps"] / serial,
                                          frac_of_overlapped=per[prec]["mpps"] / min(k1_mpps, k2_mpps))
        log(f"[bench] {prec}: {per[prec]['mpps']:.0f} Mpps, mlp {k1:.3f} ms, search {k23:.3f} ms, "
            f"probes/pkt {per[prec]['probes_per_pkt']:.2f}, filter checks/pkt {F:.2f}, "
            f"wave filter batches {per[prec]['wave_rounds']:.2f}, wave probe steps {per[prec]['wave_steps']:.2f}")

    probe_all = None
    if not args.skip_probe_all:
        T.tang_model_unload(rs)
        pst = T.tang_classify(rs, d_hdr, d_out, n, stream, want_stats=True)
        assert np.array_equal(d_out.cpu().numpy().view(np.uint32), got_by_prec[args.precisions.split(",")[0]])
        for _ in range(args.warmup):
            T.tang_classify(rs, d_hdr, d_out, n, stream)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(args.steps):
            T.tang_classify(rs, d_hdr, d_out, n, stream)
        torch.cuda.synchronize()
        probe_all = {"mpps": n * args.steps / (time.perf_counter() - w0) / 1e6,
                     "probes_per_pkt": pst["probes"] / n, "records_per_pkt": pst["records"] / n}
        log(f"[bench] no model (every tuple, best-key order): {probe_all['mpps']:.0f} Mpps")

    # the same answers in every precision; sample checked against the oracle below
    base = args.precisions.split(",")[0]
    for p, g in got_by_prec.items():
        assert np.array_equal(g, got_by_prec[base]), f"{p} answers differ from {base}"
    cand_change = None
    if "fp32" in per:
        T.tang_model_load(rs, Ws, bs, "fp32", topk=1)
        T.tang_predict(rs, d_hdr, d_out, n, stream)
        c32 = d_out.cpu().numpy().view(np.uint32) & 0xFF
        cand_change = {}
        for p in per:
            if p == "fp32":
                continue
            T.tang_model_load(rs, Ws, bs, p, topk=1, act_scales=sc if p == "fp8" else None)
            T.tang_predict(rs, d_hdr, d_out, n, stream)
            cand_change[p] = float(np.mean((d_out.cpu().numpy().view(np.uint32) & 0xFF) != c32))

    lit = None
    if not args.skip_literal and args.ordering == "specificity":
        lrules = synth.make_rules(cfg["n_rules"], seed=cfg["seed"], ordering="literal")
        lhdr = synth.make_packets(lrules, n, seed=cfg["seed"] + 1, frac_in=cfg["frac_in"], zipf_s=cfg["zipf"])
        lrs = T.tang_ruleset_create(0, lrules)
        lWs, lbs, lsc, lacc = train.fit(lrs, lrules, lhdr[: 1 << 18], H, steps=args.train_steps // 2,
                                        seed=2, device="cuda")
        T.tang_model_load(lrs, lWs, lbs, base, topk=1, act_scales=lsc if base == "fp8" else None)
        ld = torch.from_numpy(lhdr.view(np.uint8).reshape(-1)).to(dev)
        lst = T.tang_classify(lrs, ld, d_out, n, stream, want_stats=True)
        for _ in range(args.warmup):
            T.tang_classify(lrs, ld, d_out, n, stream)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(args.steps):
            T.tang_classify(lrs, ld, d_out, n, stream)
        torch.cuda.synchronize()
        lwall = time.perf_counter() - w0
        lit = {"mpps": n * args.steps / lwall / 1e6, "precision": base,
               "probes_per_pkt": lst["probes"] / n, "records_per_pkt": lst["records"] / n}
        lgot = d_out.cpu().numpy().view(np.uint32).copy()
        T.tang_ruleset_destroy(lrs)
        del ld
        log(f"[bench] literal ordering: {lit['mpps']:.0f} Mpps")

    configs = None
    if not args.skip_configs:
        T.tang_model_load(rs, Ws, bs, base, topk=1, act_scales=sc if base == "fp8" else None)
        configs = other_configs(args, rules, rs, d_hdr, base)

    hybrid = None
    if not args.skip_hybrid:
        T.tang_model_load(rs, Ws, bs, "bf16", topk=1)
        hybrid = bench_hybrid(rs, hdr, d_hdr, got_by_prec[base])

    stats = None
    if not args.skip_stats:
        stats = paper_statistics(args, rules, rs, hdr, d_hdr, d_out, got_by_prec[base], C)

    resnet = None
    if not args.skip_resnet:
        resnet = bench_resnet(args, rs, d_hdr, d_out, got_by_prec[base], C)

    # the update stream (c4), the serving loop (c5) and the drift experiment (c6), each on
    # its own rulesets; the headline ruleset's buffers are released first
    upd = srv = drift = None
    if not (args.skip_updates and args.skip_serving and args.skip_drift):
        T.tang_model_unload(rs)
        torch.cuda.empty_cache()
    if not args.skip_updates:
        upd = bench_updates(args)
        log(f"[bench] c4: lookups {upd['lookup_mpps']['mean']:.0f} Mpps, update p50 "
            f"{upd['update_ms']['p50']:.2f} ms p99 {upd['update_ms']['p99']:.2f} ms, "
            f"{upd['bit_exact']['mismatches']} mismatches of {upd['bit_exact']['checked']}")
    if not args.skip_serving:
        srv = bench_serving(args)
    if not args.skip_drift:
        drift = bench_drift(args)

    # oracle: CPU baseline on a bounded seeded sample, and the bit-exact check
    cpu = None
    exact = None
    if not args.skip_cpu:
        from oracle import oracle as orc
        samp = np.sort(np.random.default_rng(9).choice(n, min(args.cpu_sample, n), replace=False))
        threads = orc.default_threads()
        t0 = time.perf_counter()
        want = orc.classify(rules, hdr[samp], threads=threads)
        el = time.perf_counter() - t0
        s1 = samp[:20_000]
        t0 = time.perf_counter()
        orc.classify(rules, hdr[s1], threads=1)
        el1 = time.perf_counter() - t0
        cpu = {"value": len(samp) / el / 1e6, "unit": "Mpps", "cores": threads, "kind": "oracle",
               "sample": f"{len(samp)} of the {n} headers (seeded), same 524,288-rule ruleset; "
                         f"linear scan in (priority, id) order, {el:.1f}s wall",
               "one_thread_mpps": len(s1) / el1 / 1e6, "cpu_model": cpu_model()}
        mism = {p: int((g[samp] != want).sum()) for p, g in got_by_prec.items()}
        exact = {"sample": int(len(samp)), "mismatches": mism,
                 "bit_exact": all(v == 0 for v in mism.values())}
        if lit is not None:
            lw = orc.classify(lrules, lhdr[samp], threads=threads)
            lit["sample_mismatches"] = int((lgot[samp] != lw).sum())
        log(f"[bench] oracle {cpu['value']:.4f} Mpps on {threads} threads; mismatches {mism}")

    head = per.get("bf16") or per[base]
    head_prec = "bf16" if "bf16" in per else base
    dom = "k_mlp" if head["k_mlp_ms"] >= head["k_classify_ms"] else "k_classify"
    wl = "c3_512k_zipf_16m"
    if dom == "k_mlp":
        roof = {"kernel": "k_mlp", "bound": "mfma", "achieved": head["mlp_tflops"],
                "peak": PEAK_TFLOPS[head_prec], "unit": "TFLOP/s", "frac": head["mlp_frac"],
                "traffic": measured_traffic("k_mlp", wl)}
    else:
        roof = {"kernel": "k_classify", "bound": "hbm", "achieved": head["search_gbs"],
                "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": head["search_gbs"] / PEAK_HBM_GBS,
                "traffic": measured_traffic("k_classify", wl)}
    other = {"k_mlp": {"bound": "mfma", "achieved_tflops": head["mlp_tflops"], "frac": head["mlp_frac"],
                       "ms": head["k_mlp_ms"], "flop_per_pkt": flop_pkt},
             "k_classify": {"bound": "hbm", "achieved_gbs": head["search_gbs"],
                            "frac": head["search_gbs"] / PEAK_HBM_GBS, "ms": head["k_classify_ms"],
                            "bytes_per_pkt": head["search_bytes_per_pkt"],
                            "overhead_bytes_per_pkt": head["search_overhead_bytes_per_pkt"],
                            "overhead": "bucket-filter blocks (8 B each) and the predictor's "
                                        "candidate word (4 B), not counted in bytes_per_pkt",
                            "what_binds": "issue, not HBM: the whole-batch search keeps the "
                                          "texture data units about 97% busy and issues VALU "
                                          "in about 93% of its cycles (derived shares in "
                                          "profiles/k_classify_c3_512k_zipf_16m.txt)"}}
    tr = measured_traffic("k_classify", wl)
    if tr:
        other["k_classify"]["traffic_over_algorithmic"] = tr / (head["search_bytes_per_pkt"] * n)
    # the search's random accesses (filter words, slots, records: one line each) per second,
    # beside a plain library gather over a table of the same size
    acc_pkt = head["filter_checks_per_pkt"] + head["slots_per_pkt"] + head["records_per_pkt"]
    rnd = {"search_random_accesses_per_pkt": acc_pkt,
           "search_random_accesses_per_s": acc_pkt * n / (head["k_classify_ms"] * 1e-3)}
    try:
        rnd["library_gather"] = library_gather(dev, table_bytes)
        rnd["search_vs_library_gather"] = (rnd["search_random_accesses_per_s"]
                                           / rnd["library_gather"]["gathers_per_s"])
        log(f"[bench] search {rnd['search_random_accesses_per_s'] / 1e9:.1f} G random accesses/s "
            f"({acc_pkt:.2f} per header); torch gather over {rnd['library_gather']['table_bytes']} B: "
            f"{rnd['library_gather']['gathers_per_s'] / 1e9:.1f} G/s")
    except Exception as ex:  # a reference figure only: never costs the bench line
        rnd["library_gather"] = None
        log(f"[bench] library gather reference failed: {ex}")
    other["k_classify"]["random_access"] = rnd
    line = {
        "metric": "Mpps classified at 512k rules (1 MI355X)",
        "value": head["mpps"], "unit": "Mpps", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": head_prec, "data": "synthetic",
        "config": {"workload": "c3_512k: 524,288 rules (specificity order), 16,777,216 headers "
                               "Zipf(1) rule-sampled, MLP 104-256-256-C",
                   "rules": len(rules), "batch": n, "tuples": C, "ordering": args.ordering,
                   "precision": head_prec, "topk": 1},
        "latency_ms": {"p50": head["p50_ms"], "p99": head["p99_ms"], "batch": n},
        "bit_exact": exact,
        "roofline": roof, "kernels": other,
        "per_precision": per, "candidate_change_vs_fp32": cand_change,
        "literal_ordering": lit, "no_model_probe_all": probe_all, "other_configs": configs,
        "paper_resnet_predictor": resnet, "paper_statistics": stats, "paper_cpu_gpu_split": hybrid,
        "c4_updates": upd, "c5_serving": srv, "c6_drift": drift,
        "build_s": build_s, "train_top1": acc,
        "cpu_baseline": cpu,
        "paper_context": "TaNG reports 10.98 Mpps average at 512k rules (12 ClassBench-ng rulesets, "
                         "RTX 3090 + EPYC 7542, CPU-GPU hybrid); different hardware and workload",
    }
    print(json.dumps(line), flush=True)
    T.tang_ruleset_destroy(rs)



def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_classify(T, rs, d_hdr, d_out, n, reps):
    """Mean ms of tang_classify over `reps` launches after 3 warm-ups (HIP events)."""
    import torch
    s = torch.cuda.current_stream()
    for _ in range(3):
        T.tang_classify(rs, d_hdr, d_out, n, s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        T.tang_classify(rs, d_hdr, d_out, n, s)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def other_configs(args, rules3, rs3, d_hdr3, prec3):
    """The 1k-rule (FP32, 104-128-128-C) and 64k-rule wildcard-mix (FP32 vs BF16) workloads,
    and the 512k ruleset with 80% rule-sampled headers: Mpps, probes per header, answers
    against the oracle (all of them at 1k, a seeded sample otherwise), and at 64k the
    share of headers whose BF16 candidate differs from the FP32 one."""
    import numpy as np
    import torch

    from oracle import oracle as orc
    from paper_2601_03187_amd import synth, train
    from paper_2601_03187_amd import tang as T

    res = {}
    for name, precs in (("c1_1k", ("fp32",)), ("c2_64k", ("fp32", "bf16"))):
        cfg = synth.CONFIGS[name]
        rules = synth.make_rules(cfg["n_rules"], seed=cfg["seed"], ordering="specificity", mix=cfg["mix"])
        hdr = synth.make_packets(rules, cfg["n_pkts"], seed=cfg["seed"] + 1, frac_in=cfg["frac_in"])
        n = len(hdr)
        rs = T.tang_ruleset_create(0, rules)
        Ws, bs, sc, acc = train.fit(rs, rules, hdr[:200_000], cfg["hidden"], steps=500, seed=1,
                                    device="cuda")
        d_hdr = torch.from_numpy(hdr.view(np.uint8).reshape(-1)).cuda()
        d_out = torch.empty(n, dtype=torch.int32, device="cuda")
        samp = np.arange(n) if n <= 10_000 else np.sort(np.random.default_rng(11).choice(n, 100_000, replace=False))
        want = orc.classify(rules, hdr[samp])
        out = {"rules": len(rules), "headers": n, "hidden": cfg["hidden"], "train_top1": acc}
        cands = {}
        for p in precs:
            T.tang_model_load(rs, Ws, bs, p, topk=1)
            st = T.tang_classify(rs, d_hdr, d_out, n, torch.cuda.current_stream(), want_stats=True)
            got = d_out.cpu().numpy().view(np.uint32)
            ms = time_classify(T, rs, d_hdr, d_out, n, 50 if n <= 10_000 else 20)
            T.tang_predict(rs, d_hdr, d_out, n, torch.cuda.current_stream())
            cands[p] = d_out.cpu().numpy().view(np.uint32) & 0xFF
            out[p] = {"mpps": n / ms / 1e3, "ms_per_batch": ms, "probes_per_pkt": st["probes"] / n,
                      "records_per_pkt": st["records"] / n, "fallback_rate": st["fallbacks"] / n,
                      "oracle_checked": int(len(samp)), "mismatches": int((got[samp] != want).sum())}
        if "bf16" in cands:
            out["candidate_change_bf16_vs_fp32"] = float(np.mean(cands["bf16"] != cands["fp32"]))
        res[name] = out
        T.tang_ruleset_destroy(rs)
        del d_hdr, d_out
        log(f"[bench] {name}: " + ", ".join(f"{p} {out[p]['mpps']:.0f} Mpps ({out[p]['mismatches']} "
                                             f"mismatches of {out[p]['oracle_checked']})" for p in precs))
    cfg = synth.CONFIGS["c3_512k"]
    n = cfg["n_pkts"]
    hdr = synth.make_packets(rules3, n, seed=cfg["seed"] + 7, frac_in=0.8, zipf_s=cfg["zipf"])
    d_hdr = torch.from_numpy(hdr.view(np.uint8).reshape(-1)).cuda()
    d_out = torch.empty(n, dtype=torch.int32, device="cuda")
    st = T.tang_classify(rs3, d_hdr, d_out, n, torch.cuda.current_stream(), want_stats=True)
    got = d_out.cpu().numpy().view(np.uint32)
    samp = np.sort(np.random.default_rng(12).choice(n, 20_000, replace=False))
    want = orc.classify(rules3, hdr[samp])
    ms = time_classify(T, rs3, d_hdr, d_out, n, args.steps)
    res["c3_512k_80pct_inside"] = {"precision": prec3, "mpps": n / ms / 1e3, "ms_per_batch": ms,
                                   "probes_per_pkt": st["probes"] / n, "no_match_rate": st["no_match"] / n,
                                   "oracle_checked": int(len(samp)),
                                   "mismatches": int((got[samp] != want).sum())}
    log(f"[bench] c3 with 80% rule-sampled headers: {res['c3_512k_80pct_inside']['mpps']:.0f} Mpps")
    del d_hdr, d_out
    res["c7_wide"] = bench_wide(args, "c7_wide")
    res["c8_all_lengths"] = bench_wide(args, "c8_all_lengths")
    return res


def bench_wide(args, name):
    """A wide tuple space, 524,288 rules and 16M Zipf headers: c7_wide, 144 (SIP, DIP)
    signatures (12 prefix lengths per field); c8_all_lengths, 387 signatures over every
    prefix length 0..32 (the size of the paper's largest tuple spaces). No model, and a
    trained 104-256-256-C MLP in BF16 and FP8 (top-1). Mpps, probes per header, and a
    seeded 20,000-header oracle sample."""
    import numpy as np
    import torch

    from oracle import oracle as orc
    from paper_2601_03187_amd import synth, train
    from paper_2601_03187_amd import tang as T

    cfg = synth.CONFIGS[name]
    rules = synth.make_rules(cfg["n_rules"], seed=cfg["seed"], wide=name == "c7_wide",
                             all_lengths=name == "c8_all_lengths")
    n = cfg["n_pkts"]
    hdr = synth.make_packets(rules, n, seed=cfg["seed"] + 1, frac_in=cfg["frac_in"], zipf_s=cfg["zipf"])
    rs = T.tang_ruleset_create(0, rules)
    C = T.tang_ruleset_num_tuples(rs)
    d_hdr = torch.from_numpy(hdr.view(np.uint8).reshape(-1)).cuda()
    d_out = torch.empty(n, dtype=torch.int32, device="cuda")
    samp = np.sort(np.random.default_rng(13).choice(n, 20_000, replace=False))
    want = orc.classify(rules, hdr[samp])
    out = {"rules": len(rules), "tuples": C, "headers": n, "hidden": cfg["hidden"]}

    def run(what):
        st = T.tang_classify(rs, d_hdr, d_out, n, torch.cuda.current_stream(), want_stats=True)
        got = d_out.cpu().numpy().view(np.uint32)
        ms = time_classify(T, rs, d_hdr, d_out, n, args.steps)
        out[what] = {"mpps": n / ms / 1e3, "ms_per_batch": ms, "probes_per_pkt": st["probes"] / n,
                     "records_per_pkt": st["records"] / n, "top1_hit_rate": st["top1_hits"] / n,
                     "fallback_rate": st["fallbacks"] / n, "oracle_checked": int(len(samp)),
                     "mismatches": int((got[samp] != want).sum())}
        log(f"[bench] {name} ({C} tuples) {what}: {out[what]['mpps']:.0f} Mpps, "
            f"{out[what]['probes_per_pkt']:.2f} probes/pkt, {out[what]['mismatches']} mismatches")

    run("no_model")
    Ws, bs, sc, acc = train.fit(rs, rules, hdr[:200_000], cfg["hidden"], steps=args.train_steps,
                                seed=1, device="cuda")
    out["train_top1"] = acc
    for p in ("bf16", "fp8"):
        T.tang_model_load(rs, Ws, bs, p, topk=1, act_scales=sc if p == "fp8" else None)
        run(p)
    T.tang_ruleset_destroy(rs)
    return out


def bench_hybrid(rs, hdr, d_hdr, want):
    """The paper's own split (Sec. 5.1.2) as a comparison: the GPU predicts (BF16 model)
    chunk k + 1 and copies its candidates to pinned host memory while host threads run the
    search of chunk k (tang_search_host), on the first 4,194,304 headers of the 512k
    workload; the paper's search (a lower-priority match in the predicted tuple is kept)
    and the exact one (ordered search always). Mpps over the whole pipeline, and the share
    of answers equal to the exact ones."""
    import concurrent.futures as cf

    import numpy as np
    import torch

    from oracle import oracle as orc
    from paper_2601_03187_amd import tang as T

    n, chunk = 1 << 22, 1 << 20
    threads = orc.default_threads()
    s = torch.cuda.current_stream()
    d_cand = torch.empty(n, dtype=torch.int32, device="cuda")
    h_cand = torch.empty(n, dtype=torch.int32, pin_memory=True)
    out = np.empty(n, dtype=np.uint32)
    res = {"headers": n, "chunk": chunk, "host_threads": threads}
    with cf.ThreadPoolExecutor(1) as ex:
        for mode, exact in (("paper_search", False), ("exact_search", True)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pend = None
            for base in range(0, n, chunk):
                T.tang_predict(rs, d_hdr[16 * base:], d_cand[base:], chunk, s)
                h_cand[base:base + chunk].copy_(d_cand[base:base + chunk], non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(s)
                ev.synchronize()
                if pend is not None:
                    pend.result()
                cv = h_cand[base:base + chunk].numpy().view(np.uint32)
                pend = ex.submit(T.tang_search_host, rs, hdr[base:base + chunk], cv, 1, threads, exact,
                                 out[base:base + chunk])
            pend.result()
            el = time.perf_counter() - t0
            res[mode] = {"mpps": n / el / 1e6, "agree_with_exact": float(np.mean(out == want[:n]))}
            log(f"[bench] CPU-GPU split, {mode}: {res[mode]['mpps']:.1f} Mpps on {threads} host threads, "
                f"answers equal to the exact ones: {res[mode]['agree_with_exact']:.5f}")
    return res


def paper_statistics(args, rules, rs, hdr, d_hdr, d_out, want, C):
    """Analogue of the paper's statistics tables (Sec. 7.5) on the 512k workload, for the
    plain predictor and the paper's residual network, each trained with the paper's loop
    (alpha oversampling, beta = 0.95, rounds of epochs; reduced epochs) on the first
    1,048,576 headers: model accuracy (top-1 tuple = tuple of the exact answer) on the last
    1,048,576 headers (held out); classification accuracy of the paper's own search (the
    best rule of the predicted tuple if one matches, else the ordered search over the other
    tuples, without certification) on a seeded sample of 20,000 held-out headers, from the
    oracle restricted to each predicted tuple; this library's accuracy (its answers equal
    the oracle's); tuples; and memory accesses per lookup (filter words, slots, records)."""
    import numpy as np
    import torch

    from oracle import oracle as orc
    from paper_2601_03187_amd import train
    from paper_2601_03187_amd import tang as T

    n = len(hdr)
    ntr = 1 << 20
    held = np.arange(n - ntr, n)
    tup_of_rule = train.tuple_labels(rs, rules, rules["id"])
    label = train.tuple_labels(rs, rules, want[held])
    samp = np.sort(np.random.default_rng(13).choice(held, 20_000, replace=False))
    truth = want[samp]
    out = {"tuples": C}
    s = torch.cuda.current_stream()
    for arch, width, kw in (("mlp", 256, {}), ("resnet", 512, {"n_blocks": 6})):
        t0 = time.time()
        Ws, bs, info = train.train_paper(rs, rules, hdr[:ntr], arch=arch, hidden=width, alpha=1000,
                                         beta=0.95, rounds=3, epochs=10, device="cuda",
                                         rule_ids=want[:ntr], **kw)
        if arch == "mlp":
            T.tang_model_load(rs, Ws, bs, "bf16", topk=1)
        else:
            T.tang_model_load_resnet(rs, Ws, bs, "bf16", topk=1)
        cand = torch.empty(n, dtype=torch.int16, device="cuda")
        T.tang_mlp_forward(rs, d_hdr, n, None, cand, s)
        pred = cand.cpu().numpy().view(np.uint16).astype(np.int64)
        ok = label >= 0
        model_acc = float(np.mean(pred[held][ok] == label[ok]))
        # the paper's search: best match inside the predicted tuple, else the true answer
        # (the ordered search over the remaining tuples finds the best of them)
        paper = truth.copy()
        ps = pred[samp]
        for t in np.unique(ps):
            g = ps == t
            inside = orc.classify(rules, hdr[samp[g]], live=(tup_of_rule == t).astype(np.uint8))
            paper[g] = np.where(inside != orc.NO_MATCH, inside, truth[g])
        st = T.tang_classify(rs, d_hdr, d_out, n, s, want_stats=True)
        exact = bool(np.array_equal(d_out.cpu().numpy().view(np.uint32), want))
        out[arch] = {"train_rounds": info["rounds"], "converged": info["converged"],
                     "train_s": time.time() - t0, "model_accuracy_heldout": model_acc,
                     "paper_search_accuracy": float(np.mean(paper == truth)),
                     "this_library_accuracy": 1.0 if exact else float(np.mean(d_out.cpu().numpy().view(np.uint32) == want)),
                     "filter_words_per_lookup": st["filter_checks"] / n,
                     "slots_per_lookup": st["slots"] / n, "records_per_lookup": st["records"] / n,
                     "probes_per_lookup": st["probes"] / n}
        log(f"[bench] paper loop, {arch}: model accuracy {model_acc:.4f}, paper search accuracy "
            f"{out[arch]['paper_search_accuracy']:.5f}, exact {exact}, rounds {len(info['rounds'])}")
    out["loop_to_beta_1k"] = paper_loop_small(args)
    return out


def paper_loop_small(args):
    """The paper's training loop (Sec. 6.2) run until it reaches beta, on a ruleset a model
    of this size can learn: the 1,024-rule workload (104-128-128-C MLP), 200,000 training
    headers, alpha from 1,000, beta = 0.95, at most 5 rounds of 20 epochs. Reports every
    round's alpha, sample count and accuracy, whether beta was reached, the model's accuracy
    on 100,000 held-out headers, and that classification with it stays exact."""
    import numpy as np
    import torch

    from oracle import oracle as orc
    from paper_2601_03187_amd import synth, train
    from paper_2601_03187_amd import tang as T

    cfg = synth.CONFIGS["c1_1k"]
    rules = synth.make_rules(cfg["n_rules"], seed=cfg["seed"], ordering="specificity", mix=cfg["mix"])
    hdr = synth.make_packets(rules, 300_000, seed=cfg["seed"] + 2, frac_in=cfg["frac_in"])
    want = orc.classify(rules, hdr)
    rs = T.tang_ruleset_create(0, rules)
    try:
        t0 = time.time()
        Ws, bs, info = train.train_paper(rs, rules, hdr[:200_000], arch="mlp", hidden=cfg["hidden"],
                                         alpha=1000, beta=0.95, rounds=5, epochs=20, device="cuda",
                                         rule_ids=want[:200_000])
        train_s = time.time() - t0
        T.tang_model_load(rs, Ws, bs, "fp32", topk=1)
        held = hdr[200_000:]
        n = len(held)
        d_hdr = torch.from_numpy(held.view(np.uint8).reshape(-1).copy()).cuda()
        cand = torch.empty(n, dtype=torch.int16, device="cuda")
        T.tang_mlp_forward(rs, d_hdr, n, None, cand, torch.cuda.current_stream())
        pred = cand.cpu().numpy().view(np.uint16).astype(np.int64)
        label = train.tuple_labels(rs, rules, want[200_000:])
        ok = label >= 0
        d_out = torch.empty(n, dtype=torch.int32, device="cuda")
        T.tang_classify(rs, d_hdr, d_out, n, torch.cuda.current_stream())
        exact = bool(np.array_equal(d_out.cpu().numpy().view(np.uint32), want[200_000:]))
        res = {"rules": len(rules), "tuples": T.tang_ruleset_num_tuples(rs), "hidden": cfg["hidden"],
               "train_headers": 200_000, "epochs_per_round": 20, "rounds": info["rounds"],
               "converged": info["converged"], "train_s": train_s,
               "model_accuracy_heldout": float(np.mean(pred[ok] == label[ok])),
               "classification_exact": exact}
        log(f"[bench] paper loop to beta, 1k rules: rounds {len(info['rounds'])}, converged "
            f"{info['converged']}, held-out accuracy {res['model_accuracy_heldout']:.4f}")
        return res
    finally:
        T.tang_ruleset_destroy(rs)


def bench_resnet(args, rs, d_hdr, d_out, want, C):
    """The paper's own predictor size (7 chunks -> 512 -> 6 residual blocks -> C, BF16,
    random weights: speed only) on the first 4,194,304 headers of the 512k workload: the
    predictor alone (tang_predict, HIP events) and whole classification (chunked, two
    streams); the answers must equal the BF16 run's."""
    import numpy as np
    import torch

    from paper_2601_03187_amd import tang as T

    n = 1 << 22
    rng = np.random.default_rng(77)
    width, nb = 512, 6
    Ws = [rng.normal(0, 2.0, (width, 7))] + [rng.normal(0, 1 / np.sqrt(width), (width, width))
                                              for _ in range(2 * nb)] + [rng.normal(0, 1 / np.sqrt(width), (C, width))]
    bs = [rng.normal(0, 0.05, w.shape[0]) for w in Ws]
    T.tang_model_load_resnet(rs, Ws, bs, "bf16", topk=1)
    s = torch.cuda.current_stream()
    T.tang_predict(rs, d_hdr, d_out, n, s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    e0.record(s)
    for _ in range(reps):
        T.tang_predict(rs, d_hdr, d_out, n, s)
    e1.record(s)
    torch.cuda.synchronize()
    mlp_ms = e0.elapsed_time(e1) / reps
    flop = 2 * (7 * width + 2 * nb * width * width + width * C)
    T.tang_classify(rs, d_hdr, d_out, n, s)
    torch.cuda.synchronize()
    ok = bool(np.array_equal(d_out[:n].cpu().numpy().view(np.uint32), want[:n]))
    ms = time_classify(T, rs, d_hdr, d_out, n, reps)
    tflops = flop * n / (mlp_ms * 1e-3) / 1e12
    # for scale: the vendor library's GEMM (torch -> hipBLASLt) on one residual layer's shape
    # ([65,536 x 512] x [512 x 512], BF16), with the bias and without the residual / ReLU
    m = 1 << 16
    X = torch.randn(m, width, device="cuda", dtype=torch.bfloat16)
    W = torch.randn(width, width, device="cuda", dtype=torch.bfloat16)
    b = torch.randn(width, device="cuda", dtype=torch.bfloat16)
    for _ in range(3):
        torch.nn.functional.linear(X, W, b)
    e0.record(s)
    for _ in range(20):
        torch.nn.functional.linear(X, W, b)
    e1.record(s)
    torch.cuda.synchronize()
    lib_ms = e0.elapsed_time(e1) / 20
    del X, W, b
    res = {"headers": n, "blocks": nb, "width": width, "precision": "bf16", "weights": "random",
           "flop_per_pkt": flop, "predict_ms": mlp_ms, "predict_mpps": n / mlp_ms / 1e3,
           "predict_tflops": tflops, "predict_frac_of_bf16_peak": tflops / PEAK_TFLOPS["bf16"],
           "classify_ms": ms, "classify_mpps": n / ms / 1e3, "answers_equal_bf16_run": ok,
           "library_gemm_one_layer": {"shape": "65536 x 512 x 512, bf16, bias", "us": lib_ms * 1e3,
                                      "tflops": 2 * m * width * width / (lib_ms * 1e-3) / 1e12}}
    log(f"[bench] residual predictor (6 x 512): predict {res['predict_mpps']:.0f} Mpps "
        f"({tflops:.0f} TFLOP/s), classify {res['classify_mpps']:.0f} Mpps, answers equal: {ok}")
    return res


def bench_drift(args):
    """c6: the paper's dynamic experiment (Sec. 7.4) on one GPU. 65,536 rules; 10 windows,
    each deleting 2,000 live rules and inserting 2,000 with a SIP prefix length (4) the
    tuple set lacks (restricted insertion puts them in coarser tuples), then classifying 1M headers
    drawn from the live rules (BF16 predictor). Run twice on the same stream: immediate
    updates only, and with the deferred update (tau 5%; theta 2,500 coarse rules, the
    paper's 10,000 per 256k rules scaled): incremental training fine-tunes the model on
    fresh labels, full retraining rebuilds the tuple space from the exported live rules.
    Per window: Mpps, probes per header, the action taken; answers on a seeded sample
    against the oracle's scan of the live rules."""
    import numpy as np
    import torch

    from oracle import oracle as orc
    from paper_2601_03187_amd import synth, train
    from paper_2601_03187_amd import tang as T
    from paper_2601_03187_amd.deferred import DeferredUpdate

    cfg = synth.CONFIGS["c6_drift"]
    rules0 = synth.make_rules(cfg["n_rules"], seed=cfg["seed"], ordering="specificity")
    stream = synth.make_update_stream(rules0, cfg["windows"], cfg["per_window"], seed=cfg["seed"] + 1,
                                      prio_range=len(rules0), sip_lengths=cfg["sip_lengths"])
    n = cfg["n_pkts"]
    d_out = torch.empty(n, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()

    def train_on(rs, live, seed, init=None, epochs=4):
        h = synth.make_packets(live, 1 << 19, seed=seed, frac_in=cfg["frac_in"])
        Ws, bs, info = train.train_paper(rs, live, h, hidden=cfg["hidden"], alpha=1000, beta=0.0,
                                         rounds=1, epochs=epochs, device="cuda", init=init)
        T.tang_model_load(rs, Ws, bs, "bf16", topk=1)
        return Ws, bs

    res = {}
    for mode in ("immediate_only", "with_deferred"):
        rs = T.tang_ruleset_create(0, rules0)
        model = train_on(rs, rules0, cfg["seed"] + 2, epochs=8)
        pol = DeferredUpdate(tau=0.05, theta=2_500)
        rows, mism = [], 0
        for w in range(cfg["windows"] + 1):
            if w > 0:
                ins, dels = stream[w - 1]
                T.tang_delete(rs, dels)
                T.tang_insert(rs, ins)
            live = T.tang_ruleset_export(rs)
            hdr = synth.make_packets(live, n, seed=cfg["seed"] + 100 + w, frac_in=cfg["frac_in"])
            d_hdr = torch.from_numpy(hdr.view(np.uint8).reshape(-1)).cuda()
            st = T.tang_classify(rs, d_hdr, d_out, n, s, want_stats=True)
            got = d_out.cpu().numpy().view(np.uint32)
            samp = np.random.default_rng(w).choice(n, 2000, replace=False)
            mism += int((got[samp] != orc.classify(live, hdr[samp])).sum())
            ms = time_classify(T, rs, d_hdr, d_out, n, 10)
            mpps = n / ms / 1e3
            coarse = T.tang_ruleset_coarse_rules(rs)
            action = pol.observe(mpps, coarse) if mode == "with_deferred" else None
            if action == "incremental":
                model = train_on(rs, live, cfg["seed"] + 200 + w, init=model, epochs=2)
            elif action == "full":
                T.tang_ruleset_destroy(rs)
                rs = T.tang_ruleset_create(0, live)
                model = train_on(rs, live, cfg["seed"] + 300 + w, epochs=8)
            if action:
                pol.deployed(action)
            rows.append({"window": w, "mpps": mpps, "probes_per_pkt": st["probes"] / n,
                         "records_per_pkt": st["records"] / n,
                         "fallback_rate": st["fallbacks"] / n, "coarse_rules": coarse,
                         "action": action})
            log(f"[bench c6] {mode} window {w}: {mpps:.0f} Mpps, probes/pkt {st['probes'] / n:.2f}, "
                f"records/pkt {st['records'] / n:.2f}, coarse rules {coarse}, action {action}")
            del d_hdr
        T.tang_ruleset_destroy(rs)
        res[mode] = {"windows": rows, "sample_mismatches": mism}
    return res


def print_drift(res):
    import numpy as np
    line = {"metric": "c6 drifting updates: Mpps per window (1 MI355X)",
            "value": float(np.mean([r["mpps"] for r in res["with_deferred"]["windows"]])),
            "unit": "Mpps (mean over windows, with deferred update)", "n_gpus": 1,
            "higher_is_better": True, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": "c6_drift: 65,536 rules, 10 windows x (2,000 deletes + 2,000 "
                                   "inserts with SIP prefix length 4), 1M headers per window"},
            "modes": res}
    print(json.dumps(line), flush=True)


def bench_updates(args):
    """c4: the 512k ruleset under 100 rounds of (100 inserts + 100 deletes), each followed
    by a 1M-header lookup batch from the live rules; fixed BF16 weights. Per round: the
    update latency (host + device, synchronised), lookup Mpps, and answers on a seeded
    sample of the batch against the oracle's re-scan of the live rules."""
    import numpy as np
    import torch

    from oracle import oracle as orc
    from paper_2601_03187_amd import synth, train
    from paper_2601_03187_amd import tang as T

    cfg = synth.CONFIGS["c4_512k_updates"]
    rules = synth.make_rules(cfg["n_rules"], seed=cfg["seed"], ordering="specificity")
    rs = T.tang_ruleset_create(0, rules)
    h0 = synth.make_packets(rules, 1 << 18, seed=cfg["seed"] + 1, frac_in=cfg["frac_in"])
    Ws, bs, sc, acc = train.fit(rs, rules, h0, cfg["hidden"], steps=args.train_steps, seed=1, device="cuda")
    T.tang_model_load(rs, Ws, bs, "bf16", topk=1)
    ups = synth.make_update_stream(rules, args.rounds, cfg["per_round"], seed=cfg["seed"] + 2,
                                   prio_range=len(rules))
    all_rules = [rules]
    live = np.ones(len(rules), dtype=bool)
    id_pos = {int(i): k for k, i in enumerate(rules["id"])}
    n = cfg["n_pkts"]
    d_out = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    lat, mpps, mism, checked = [], [], 0, 0
    sample = args.update_sample
    h_first = synth.make_packets(rules, n, seed=cfg["seed"] + 99, frac_in=cfg["frac_in"])
    d_first = torch.from_numpy(h_first.view(np.uint8).reshape(-1)).cuda()
    st0 = T.tang_classify(rs, d_first, d_out, n, stream, want_stats=True)
    del d_first
    for rd, (ins, dels) in enumerate(ups):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        T.tang_insert(rs, ins)
        T.tang_delete(rs, dels)
        lat.append((time.perf_counter() - t0) * 1e3)
        base = sum(len(a) for a in all_rules)
        all_rules.append(ins)
        live = np.concatenate([live, np.ones(len(ins), dtype=bool)])
        for k, i in enumerate(ins["id"]):
            id_pos[int(i)] = base + k
        for i in dels:
            live[id_pos[int(i)]] = False
        cat = np.concatenate(all_rules)
        hdr = synth.make_packets(cat[live], n, seed=cfg["seed"] + 100 + rd, frac_in=cfg["frac_in"])
        d_hdr = torch.from_numpy(hdr.view(np.uint8).reshape(-1)).cuda()
        T.tang_classify(rs, d_hdr, d_out, n, stream)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        T.tang_classify(rs, d_hdr, d_out, n, stream)
        b.record(stream)
        torch.cuda.synchronize()
        mpps.append(n / a.elapsed_time(b) / 1e3)
        got = d_out.cpu().numpy().view(np.uint32)
        samp = np.random.default_rng(rd).choice(n, sample, replace=False)
        mism += int((orc.classify(cat, hdr[samp], live=live) != got[samp]).sum())
        checked += len(samp)
        if rd % 10 == 0:
            log(f"[bench c4] round {rd}: update {lat[-1]:.2f} ms, lookup {mpps[-1]:.0f} Mpps")
    st = T.tang_classify(rs, d_hdr, d_out, n, stream, want_stats=True)
    res = {"workload": "c4_512k_updates: 524,288 rules, %d rounds x (100 inserts + 100 deletes) "
                       "+ 1M-header lookups, BF16 predictor" % args.rounds,
           "rounds": args.rounds,
           "lookup_mpps": {"mean": float(np.mean(mpps)), "first": mpps[0], "last": mpps[-1],
                           "min": min(mpps), "max": max(mpps), "per_round": mpps},
           "update_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "max": max(lat),
                         "per": "100 inserts + 100 deletes, synchronised"},
           "before_updates": {"probes_per_pkt": st0["probes"] / n, "records_per_pkt": st0["records"] / n,
                              "top1_hit_rate": st0["top1_hits"] / n, "train_top1": acc},
           "last_round": {"probes_per_pkt": st["probes"] / n, "records_per_pkt": st["records"] / n,
                          "top1_hit_rate": st["top1_hits"] / n},
           "bit_exact": {"sample_per_round": sample, "checked": checked, "mismatches": mism,
                         "bit_exact": mism == 0}}
    T.tang_ruleset_destroy(rs)
    return res


def print_updates(res):
    line = {"metric": "c4 update stream at 512k rules (1 MI355X)", "value": res["lookup_mpps"]["mean"],
            "unit": "Mpps", "n_gpus": 1, "higher_is_better": True, "dtype": "bf16",
            "data": "synthetic", "config": {"workload": res["workload"]}, **res}
    print(json.dumps(line), flush=True)


def bench_serving(args):
    """c5: three device-resident rulesets (10k, 100k, 512k rules, BF16 predictors) behind
    the serving loop; requests of log-uniform size 32..65,536 with a uniform ruleset tag.
    After a warm-up burst, two bursts measure saturation (the faster one counts); then
    Poisson arrivals at 25/50/75/90% of it report
    p50/p99 request latency (submit -> results on the host) and delivered Mpps. A sample of
    requests is checked against the same headers classified alone."""
    import numpy as np
    import torch

    from paper_2601_03187_amd import synth, train
    from paper_2601_03187_amd import tang as T

    cfg = synth.CONFIGS["c5_serving"]
    sets = []
    for k, n_rules in enumerate(cfg["sizes"]):
        rules = synth.make_rules(n_rules, seed=cfg["seed"] + k, ordering="specificity")
        rs = T.tang_ruleset_create(0, rules)
        pool = synth.make_packets(rules, 1 << 21, seed=cfg["seed"] + 10 + k, frac_in=cfg["frac_in"])
        Ws, bs, sc, acc = train.fit(rs, rules, pool[: 1 << 17], cfg["hidden"], steps=args.train_steps // 2,
                                    seed=k, device="cuda")
        T.tang_model_load(rs, Ws, bs, "bf16", topk=1)
        sets.append((rules, rs, pool))
    log("[bench c5] rulesets ready")
    # batches merge requests up to 262,144 headers (four of the largest requests): the
    # fixed cost of a batch (launches, copies, a partly filled GPU) then spreads over more
    # headers when requests queue up (saturation 740 Mpps with 65,536, about 1,900 with 262,144,
    # measured); at low load a batch is a single request either way
    srv = T.tang_server_create(0, n_streams=4, max_batch=262144, use_graphs=1)
    tags = [T.tang_server_add_ruleset(srv, rs) for _, rs, _ in sets]
    for t in tags:   # every (ruleset, size class, slot) graph recorded before any request
        T.tang_server_prepare(srv, t)

    def run(n_req, rate, seed):
        t_arr, sizes, tg = synth.make_requests(n_req, len(sets), seed=seed, rate_per_s=rate or 1.0)
        rng = np.random.default_rng(seed)
        # requests (header slices and result buffers) are made before the clock starts, so
        # the submitting loop does nothing but wait for arrival times and submit; the result
        # buffers are written once here, since the first write into a fresh buffer page
        # faults, and those faults would land on the serving loop's result copies (about 17k
        # pages per level: enough to slow a whole level)
        work = []
        for q in range(n_req):
            pool = sets[tg[q]][2]
            off = int(rng.integers(0, len(pool) - sizes[q]))
            work.append((int(tg[q]), pool[off: off + sizes[q]], np.zeros(sizes[q], dtype=np.uint32)))
        for _, _, out in work:
            out.fill(0xFFFFFFFF)
        reqs = []
        t0 = time.perf_counter()
        for q, (tag, hdr, out) in enumerate(work):
            if rate:
                while time.perf_counter() - t0 < t_arr[q]:
                    pass
            reqs.append((tag, hdr, out, T.tang_server_submit(srv, tags[tag], hdr, out)))
        for _, _, _, r in reqs:
            T.tang_server_wait(r, 120_000_000)
        times = [T.tang_server_req_times(r) for *_, r in reqs]
        first = min(t[0] for t in times)
        last = max(t[2] for t in times)
        lat = [(d - s) / 1e6 for s, a, d in times]
        pk = int(sum(sizes))
        return reqs, {"requests": n_req, "packets": pk, "mpps": pk / ((last - first) / 1e9) / 1e6,
                      "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                      "offered_req_per_s": rate, "submit_s": time.perf_counter() - t0}

    run(args.requests, 0, seed=1)  # warm-up
    # two saturation bursts: a runtime copy call that holds for several milliseconds (seen
    # a few times per process) can land in one; the faster burst sets the load levels, and
    # both are reported
    sats = [run(args.requests, 0, seed=2)[1], run(args.requests, 0, seed=3)[1]]
    sat = max(sats, key=lambda r: r["mpps"])
    mean_size = sat["packets"] / sat["requests"]
    sat_rate = sat["mpps"] * 1e6 / mean_size
    levels = {}
    for frac in (0.25, 0.5, 0.75, 0.9):
        reqs, r = run(args.requests, frac * sat_rate, seed=int(frac * 100))
        levels[f"{int(frac * 100)}%"] = r
        log(f"[bench c5] load {frac:.0%}: p50 {r['p50_ms']:.3f} ms p99 {r['p99_ms']:.3f} ms, {r['mpps']:.0f} Mpps")
    bad = 0
    for tag, hdr, out, r in reqs[:50]:
        bad += int((T.tang_classify_host(sets[tag][1], hdr) != out).sum())
    for *_, r in reqs:
        T.tang_server_req_free(r)
    res = {"workload": "c5_serving: rulesets of 10k/100k/512k rules, Poisson requests, sizes "
                       "log-uniform 32..65536, 4 streams, batches up to 262,144 headers, HIP graphs, "
                       "BF16 predictors",
           "saturation": sat, "saturation_bursts_mpps": [r["mpps"] for r in sats], "loads": levels,
           "alone_vs_mix": {"requests_checked": 50, "mismatches": bad}}
    T.tang_server_destroy(srv)
    for _, rs, _ in sets:
        T.tang_ruleset_destroy(rs)
    return res


def print_serving(res):
    line = {"metric": "c5 serving: p50/p99 request latency and Mpps (1 MI355X)",
            "value": res["loads"]["75%"]["p99_ms"], "unit": "ms (p99 at 75% load)", "n_gpus": 1,
            "higher_is_better": False, "dtype": "bf16", "data": "synthetic",
            "config": {"workload": res["workload"]}, **res}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
