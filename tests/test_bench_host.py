"""Host-side logic of bench.py (no GPU): the one-GPU guard and the rule that
the committed HBM traffic figure is reported only for the kernel source and
workload it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_touching_a_device():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_kernel_source_hash_is_short_hex():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)


@pytest.mark.parametrize("same_source,same_workload", [(True, True), (False, True), (True, False)])
def test_traffic_reported_only_for_its_source_and_workload(tmp_path, monkeypatch, same_source,
                                                           same_workload):
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({
        "kernel_source_sha256_16": bench.kernel_source_hash() if same_source else "0" * 16,
        "workload": "room" if same_workload else "other",
        "hbm_bytes_per_launch": 1234.5}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    got = bench.load_traffic("room")
    assert got == (1234.5 if same_source and same_workload else None)


def test_traffic_missing_file_is_none(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.json"))
    assert bench.load_traffic("room") is None


def test_weight_bound_counts_one_weight_set_per_256_frame_block():
    # 576,000 candidates x 6,544 samples per frame x 2 frame blocks (500 frames)
    b = bench.weight_bound(576000, 6544, 500, 4.0)
    assert b["weights_per_call"] == 576000 * 6544 * 2
    # the time is weights x instructions per weight / 64 lanes / issue rate
    ms = 576000 * 6544 * 2 * bench.MX_VALU_PER_WEIGHT / 64 / (1024 * 2.4e9 / 4) * 1e3
    assert b["ms"] == pytest.approx(ms, rel=1e-12)
    assert b["frac_of_map_time"] == pytest.approx(ms / 4.0, rel=1e-12)
    # 256 frames still fit one block; 257 need two
    assert bench.weight_bound(10, 10, 256, 1.0)["weights_per_call"] == 100
    assert bench.weight_bound(10, 10, 257, 1.0)["weights_per_call"] == 200
