"""Host-side checks of the benchmark's bookkeeping (no GPU): the stored HBM
traffic counters are reported only for the machine code they were taken on,
the algorithmic FLOP count follows its stated formula, and more than one GPU
is refused with a message."""
import json
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2308_14278_amd import codeobj  # noqa: E402


def test_algorithmic_flops_formula():
    # 11 per near pair, 8 per Taylor term after a_0, 8 for map and pixel
    st = SimpleNamespace(near_pairs=900, rays=100)
    assert bench.algorithmic_flops(st, 4) == 11 * 900 + (8 * 3 + 8) * 100
    assert bench.algorithmic_flops(st, 1) == 11 * 900 + 8 * 100


def test_traffic_only_for_the_measured_machine_code(monkeypatch, tmp_path):
    rec = {"kernel_symbol": "k", "kernel_code_sha": "0123456789abcdef", "bytes_per_ray": 0.5}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    monkeypatch.setattr(codeobj, "kernel_code_sha", lambda sym, lib=None: "0123456789abcdef")
    assert bench.load_traffic(1000) == 500.0
    monkeypatch.setattr(codeobj, "kernel_code_sha", lambda sym, lib=None: "fedcba9876543210")
    assert bench.load_traffic(1000) is None
    monkeypatch.setattr(codeobj, "kernel_code_sha", lambda sym, lib=None: None)
    assert bench.load_traffic(1000) is None
    path.write_text("not json")
    assert bench.load_traffic(1000) is None


def test_stored_traffic_record_names_its_code():
    with open(bench.TRAFFIC_FILE) as f:
        rec = json.load(f)
    assert len(rec["kernel_code_sha"]) == 16 and rec["kernel_symbol"].startswith("_Z")
    assert rec["bytes"] == pytest.approx(rec["bytes_per_ray"] * rec["rays"])
    assert rec["bytes"] == pytest.approx(rec["fetch_kib"] * 1024 * rec["fetch_scale"]
                                         + rec["write_kib"] * 1024 * rec["write_scale"])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "1 GPU" in (r.stdout + r.stderr)
