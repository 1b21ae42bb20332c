"""Host-side logic of bench.py (no GPU): algorithmic byte counts of the
1024x1024x4 workload, the traffic summary's source check, and the refusal of
more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_loop_workload():
    g = (1024, 1024, 4)
    N = 1024 * 1024 * 4
    spec = 1024 * 12 * 1024 * 8                 # L = 1024 bins, 12 signals, 1024 rows, complex FP32
    tensor = 1025 * 1025 * 6 * 4 * 4            # (L+1)(Py/2+1) bins, 6 components, 4 layer offsets
    assert bench.algorithmic_bytes(g, True, "demag_xfwd") == 12 * N + spec
    assert bench.algorithmic_bytes(g, True, "demag_ypass") == 2 * spec + tensor
    assert bench.algorithmic_bytes(g, True, "demag_xinv") == spec + 6 * N
    assert bench.algorithmic_bytes(g, True, "colour_pass") == 48 * N // 2
    assert bench.algorithmic_bytes(g, False, "colour_pass") == 36 * N // 2
    per_sweep = 2 * sum(bench.algorithmic_bytes(g, True, k) for k in bench.KINDS[:5])
    assert abs(per_sweep / N - 324.1) < 0.1
    # fused colour pass: spectrum in and out, m read once, own colour written
    assert bench.algorithmic_bytes(g, True, "fused_pass") == 2 * spec + 18 * N
    fused_sweep = 2 * sum(bench.algorithmic_bytes(g, True, k) for k in ("demag_ypass", "fused_pass"))
    assert abs(fused_sweep / N - 276.1) < 0.1
    assert bench.algorithmic_bytes(g, True, "fused_pass_half") == spec + 18 * N
    half_sweep = 2 * sum(bench.algorithmic_bytes(g, True, k) for k in ("demag_xfwd", "demag_ypass", "fused_pass_half"))
    assert abs(half_sweep / N - 300.1) < 0.1


def test_counted_traffic_follows_sources(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    import hashlib
    rec = {"sources": ["k.hip"], "source_sha256": hashlib.sha256(b"kernel v1\n").hexdigest(),
           "bytes_per_launch": {"demag_ypass": {"total": 123.0}}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / bench.TRAFFIC_SOURCES_NOTE).write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counted_traffic("demag_ypass") == 123.0
    assert bench.counted_traffic("colour_pass") is None
    src.write_text("kernel v2\n")                 # kernel changed since the counters were taken
    assert bench.counted_traffic("demag_ypass") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
