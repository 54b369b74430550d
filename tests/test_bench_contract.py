"""bench.py pieces that run without a GPU: the algorithmic byte model behind the
roofline, the one-GPU guard, and the committed counter file's key."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_per_site():
    # 64 x 32 tiles: edge records (2 (64 + 32) + 16) / 2048 B and edge copies
    # (64 + 32) 16 / 2048 B per site
    rec = (2 * 96 + 16) / 2048.0
    cop = 96 * 16 / 2048.0
    assert bench.alg_bytes_per_site("bonds_ccl") == pytest.approx(8 + 2 + 0.25 + rec)
    assert bench.alg_bytes_per_site("flip") == pytest.approx(2 + 16 + cop)
    assert bench.alg_bytes_per_site("fused") == pytest.approx(2 + 16 + cop + 2 + 0.25 + rec)
    assert bench.alg_bytes_per_site("flip") == pytest.approx(18.75)
    assert bench.alg_bytes_per_site("merge") == 0.0
    # the fused launch at L = 4096 (the figure the roofline divides by its time)
    assert bench.alg_bytes_per_site("fused") * 4096 ** 2 == pytest.approx(354025472.0)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "1 GPU" in r.stderr, r.stderr


def test_counter_file_is_keyed_to_the_device_sources(tmp_path, monkeypatch):
    rec = json.load(open(bench.COUNTERS))
    assert len(rec["kernel_source_sha256"]) == 64
    # (no merge kernel runs when the tile pass unites the tile edges)
    for k in ("fused", "coins") + (("merge",) if "merge" in rec["kernels"] else ()):
        assert rec["kernels"][k]["fetch_kib"] > 0 and rec["kernels"][k]["valu_insts"] > 0
    # counters taken on other sources are not used
    stale = dict(rec, kernel_source_sha256="0" * 64)
    path = tmp_path / "counters.json"
    path.write_text(json.dumps(stale))
    monkeypatch.setattr(bench, "COUNTERS", str(path))
    assert bench.traffic_from_counters("fused", 4096 ** 2) is None
    assert bench.valu_from_counters("fused") is None
