"""The benchmark's contract on the CPU: one GPU only, the roofline peak, and
the HBM-traffic figure taken only for the kernel sources it was measured on."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_int32_peak():
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    assert abs(bench.PEAK_INT32_TOPS - 256 * 4 * 16 * 2.4e9 / 1e12) < 1e-9
    assert abs(bench.PEAK_INT32_TOPS - 39.3216) < 1e-6


def test_traffic_needs_matching_sources(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.load_traffic() is None  # no file
    f.write_text(json.dumps({"bytes_per_launch": 123, "source_hash": "0" * 16}))
    assert bench.load_traffic() is None  # counters of other sources
    f.write_text(json.dumps({"bytes_per_launch": 123,
                             "source_hash": bench.kernel_source_hash()}))
    assert bench.load_traffic() == 123


def test_committed_traffic_file_is_well_formed():
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic_c2.json")))
    for key in ("fetch_size_kib", "write_size_kib", "fetch_scale", "write_scale",
                "bytes_per_launch", "source_hash", "commands"):
        assert key in t
    want = t["fetch_size_kib"] * 1024 * t["fetch_scale"] + t["write_size_kib"] * 1024 * t["write_scale"]
    assert abs(t["bytes_per_launch"] - want) <= 1
