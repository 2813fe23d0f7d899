"""Host-side checks of the benchmark's contract (no GPU): it refuses more
than one GPU before touching the device, its counter-measured traffic of the
fused kernel belongs to the current sources, and its CPU baseline reports
the oracle in the two modes with the cores it used."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr


def test_fused_traffic_matches_the_sources():
    import bench
    assert bench.fused_source_digest() == bench.FUSED_TRAFFIC["sources_sha256"], \
        "fused kernel sources changed: re-take the FETCH_SIZE / WRITE_SIZE counters"
    assert bench.fused_traffic() == bench.FUSED_TRAFFIC["bytes"] > 0


def test_cpu_baseline_modes():
    import bench
    r = bench.cpu_baseline("grid4x4_d10_m0", budget_s=0.5, max_workers=2)
    assert r["kind"] == "oracle" and r["unit"] == "amplitudes/s"
    assert set(r["modes"]) <= {"one_process", "slices_across_processes"} and "one_process" in r["modes"]
    best = max(r["modes"].values(), key=lambda m: m["value"])
    assert r["value"] == best["value"] and r["cores"] == best["cores"]
    json.dumps(r)


def test_permute_traffic_matches_the_sources():
    import bench
    assert bench.source_digest(bench.PERMUTE_SOURCES) == bench.PERMUTE_TRAFFIC["sources_sha256"], \
        "permute kernel sources changed: re-take its FETCH_SIZE / WRITE_SIZE counters"
    assert bench.PERMUTE_TRAFFIC["bytes"] > 2 * (1 << 31)
