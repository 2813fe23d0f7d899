"""Host-side checks of the benchmark's contract (no GPU): it refuses more
than one GPU before touching the device, counter-measured figures are
reported only for the sources (and plan) they were taken on, and its CPU
baselines report the oracle in the two modes with the cores they used."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr


def test_fused_traffic_is_gated_by_the_sources(monkeypatch):
    import bench
    assert bench.FUSED_TRAFFIC["bytes"] > 0
    want = bench.FUSED_TRAFFIC["bytes"] if bench.fused_source_digest() == bench.FUSED_TRAFFIC["sources_sha256"] \
        else None
    assert bench.fused_traffic() == want
    monkeypatch.setitem(bench.FUSED_TRAFFIC, "sources_sha256", "0" * 64)
    assert bench.fused_traffic() is None


def test_headline_counters_are_gated_by_sources_and_sliced_set(monkeypatch):
    import bench
    rec = {"mfma_util": 0.1, "dominant": {"bytes": 1}, "amplitude": {"bytes": 2}}
    monkeypatch.setattr(bench, "C3_COUNTERS", {"sources_sha256": bench.step_source_digest(), "mu": [1, 2],
                                               "fp32": rec})
    assert bench.c3_counters("fp32", [1, 2]) == (rec, None)
    assert bench.c3_counters("fp32", [2, 1])[0] is None
    assert bench.c3_counters("bf16x6", [1, 2])[0] is None
    monkeypatch.setitem(bench.C3_COUNTERS, "sources_sha256", "0" * 64)
    got, why = bench.c3_counters("fp32", [1, 2])
    assert got is None and "sources" in why


def test_cpu_baseline_modes():
    import bench
    r = bench.cpu_baseline("grid4x4_d10_m0", budget_s=0.5, max_workers=2)
    assert r["kind"] == "oracle" and r["unit"] == "amplitudes/s"
    assert set(r["modes"]) <= {"one_process", "slices_across_processes"} and "one_process" in r["modes"]
    best = max(r["modes"].values(), key=lambda m: m["value"])
    assert r["value"] == best["value"] and r["cores"] == best["cores"]
    json.dumps(r)


def test_cpu_baseline_on_sampled_slices():
    import bench
    r = bench.cpu_baseline_slices("grid5x5_d16_m6", budget_s=0.5, max_workers=2)
    assert r["kind"] == "oracle" and r["unit"] == "amplitudes/s" and r["value"] > 0
    one = r["modes"]["one_process"]
    assert 1 <= one["slices"] <= 64 and one["cores"] == 1
    assert r["value"] == max(m["value"] for m in r["modes"].values())
    assert "slices 0.." in r["sample"]
    json.dumps(r)


def test_permute_traffic_is_gated_by_the_sources():
    import bench
    assert bench.PERMUTE_TRAFFIC["bytes"] > 2 * (1 << 31)
