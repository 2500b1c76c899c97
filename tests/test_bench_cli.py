"""Host-side checks of bench.py (no GPU): the one-GPU rule, and the guard
that reports the committed HBM counters only while the counted kernels'
sources are the ones they were taken from."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.join(os.path.dirname(__file__), "..")
sys.path.insert(0, ROOT)
bench = pytest.importorskip("bench")


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_is_reported_only_for_the_counted_sources(tmp_path, monkeypatch):
    """measured_traffic gives the committed counters while the hash of the
    counted kernels' sources matches the one stored with them, and None as
    soon as it does not."""
    with open(os.path.join(ROOT, "profiles", "n12d6_hbm_traffic.json")) as f:
        d = json.load(f)
    current = bench.kernel_sources_hash()
    got = bench.measured_traffic("step:k_gram_bf3")
    assert (got is not None) == (d["source_hash"] == current)
    # a stored hash that differs from the sources: no traffic
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "n12d6_hbm_traffic.json").write_text(
        json.dumps(dict(d, source_hash="0" * 16)))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: current)
    assert bench.measured_traffic("step:k_gram_bf3") is None
    # the matching hash: the stored read + write bytes
    (tmp_path / "profiles" / "n12d6_hbm_traffic.json").write_text(json.dumps(dict(d, source_hash=current)))
    v = d["kernels"]["step:k_gram_bf3"]
    assert bench.measured_traffic("step:k_gram_bf3") == v["read_bytes"] + v["write_bytes"]
