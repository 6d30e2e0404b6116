"""Host-side logic of bench.py (no GPU): the roofline object's arithmetic,
the gating of the committed traffic record on the stage kernel's sources,
the single-GPU refusal, and that the committed record matches the current
sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _run(npts=1_000_000_000, launches=100, ms_per_launch=70.0):
    return {"kernel_ms": launches * ms_per_launch, "launches": launches}


@pytest.mark.parametrize("precision,method,fused", [("fp64", 280.0, 200.0), ("fp32", 168.0, 128.0)])
def test_roofline_is_algorithmic_bytes_over_mean_launch_time(precision, method, fused):
    npts = 1_000_000_000
    r = bench.roofline(precision, False, npts, _run(npts, 100, 70.0), "no-such-workload")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["avg_launch_ms"] == 70.0
    assert r["algorithmic_bytes_per_point"] == method
    assert r["achieved"] == pytest.approx(method * npts / 0.070 / 1e9, abs=0.05)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, abs=1e-4)
    assert r["fused"]["bytes_per_point"] == pytest.approx(fused)
    assert r["traffic"] is None                      # no record for this workload
    held = bench.roofline(precision, True, npts, _run(npts, 100, 70.0), "no-such-workload")
    assert held["algorithmic_bytes_per_point"] == method + bench.HELD_VISC_BYTES[precision]


def test_traffic_record_is_current_and_gated_on_the_sources(tmp_path, monkeypatch):
    with open(bench.TRAFFIC_FILE) as fh:
        rec = json.load(fh)[bench.DOMINANT_KERNEL]
    for wl in ("big1B-fp64", "big1B-fp32"):
        assert rec[wl]["source_sha"] == bench.source_hash(), \
            f"profiles/traffic.json ({wl}) predates the stage kernel's sources"
        assert bench.traffic_for(bench.DOMINANT_KERNEL, wl) == rec[wl]["bytes_per_launch"]
    stale = {bench.DOMINANT_KERNEL: {"big1B-fp64": dict(rec["big1B-fp64"], source_sha="0" * 16)}}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.traffic_for(bench.DOMINANT_KERNEL, "big1B-fp64") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
