"""Host-side pieces of bench.py: the --gpus guard and the rule that measured
HBM traffic is reported only for the sources it was measured on."""
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
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    digest = bench.sources_digest()
    assert len(digest) == 64
    good = tmp_path / "good.txt"
    good.write_text(f"sources sha256: {digest}\ntraffic bytes per launch: 123456789\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(good))
    assert bench.measured_traffic() == 123456789
    stale = tmp_path / "stale.txt"
    stale.write_text(f"sources sha256: {'0' * 64}\ntraffic bytes per launch: 123456789\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic() is None
