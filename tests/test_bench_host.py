"""Host logic of bench.py (no GPU): the one-GPU guard, the roofline
arithmetic, and the use of the committed counter summary only while its
source hash matches the kernels."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_roofline_arithmetic():
    # 8 B/px over 1e6 px in 0.1 ms: 80 GB/s, 1 % of 8000 GB/s
    rf = bench.roofline(("k_global_rows", 0.1), 1_000_000, "c1")
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s"
    assert rf["achieved"] == pytest.approx(80.0)
    assert rf["frac"] == pytest.approx(0.01)
    assert rf["bytes_per_launch"] == 8_000_000
    assert rf["traffic"] is None                      # counters exist for the 64-frame batch only


def test_counter_summary_used_only_on_matching_sources(tmp_path, monkeypatch):
    entry = {"hbm_bytes_per_launch": 123, "valu_instr_per_launch": 1000}
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    f.write_text(json.dumps({"kernel_sha": bench.kernel_sha(), "kernels": {"k_global_rows": entry}}))
    assert bench.traffic_for("k_global_rows", "c2") == 123
    vc = bench.valu_ceiling("k_global_rows", "c2", 0.001)
    # 64 lanes x 1000 instructions in 1 us = 64 G lane-ops/s
    assert vc["bound"] == "alu" and vc["achieved"] == pytest.approx(0.06, abs=0.01)
    assert vc["frac"] == pytest.approx(64e9 / (bench.VALU_PEAK_TOPS * 1e12), rel=0.05)
    f.write_text(json.dumps({"kernel_sha": "0" * 16, "kernels": {"k_global_rows": entry}}))
    assert bench.traffic_for("k_global_rows", "c2") is None
    assert bench.valu_ceiling("k_global_rows", "c2", 0.001) is None


def test_committed_summary_names_current_kernels_or_is_ignored():
    """The committed counter summary is either taken on the current sources
    or ignored by the bench (never applied to other kernels)."""
    with open(bench.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t.get("kernel_sha") == bench.kernel_sha():
        assert bench.traffic_for("k_global_rows", "c2") == t["kernels"]["k_global_rows"]["hbm_bytes_per_launch"]
    else:
        assert bench.traffic_for("k_global_rows", "c2") is None
