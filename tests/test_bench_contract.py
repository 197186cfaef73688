"""Host-side parts of the benchmark's report: the refusal of more than one GPU, and the
rule that a kernel's measured HBM traffic is reported only while its source is the one
the counters were taken on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WL = "c3_512k_zipf_16m"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    for kernel in ("k_classify", "k_mlp"):
        with open(os.path.join(ROOT, "profiles", f"traffic_{kernel}_{WL}.json")) as f:
            t = json.load(f)
        assert t["kernel"] == kernel and t["source"] == bench.KERNEL_SOURCES[kernel]
        # HBM bytes = FETCH_SIZE and WRITE_SIZE (KiB), each scaled by its copy calibration
        cal = t["copy_calibration"]
        want = 1024 * (t["fetch_size_kib"] * cal["fetch_scale"] + t["write_size_kib"] * cal["write_scale"])
        assert abs(t["traffic_bytes_per_launch"] - want) <= 1e-6 * want
        assert abs(cal["fetch_scale"] - cal["bytes"] / 1024 / cal["fetch_size_kib"]) < 1e-9
        # a matching source reports the figure, a changed one reports nothing
        monkeypatch.setitem(bench.KERNEL_SOURCES, kernel, t["source"])
        if bench.source_sha(t["source"]) == t["source_sha"]:
            assert bench.measured_traffic(kernel, WL) == t["traffic_bytes_per_launch"]
        other = tmp_path / f"{kernel}.hip"
        other.write_text("// another kernel\n")
        monkeypatch.setitem(bench.KERNEL_SOURCES, kernel, str(other))
        assert bench.measured_traffic(kernel, WL) is None
    assert bench.measured_traffic("k_classify", "no_such_workload") is None
