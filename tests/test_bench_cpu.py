"""Host-side pieces of the benchmark: the one-GPU contract, the traffic
record's validity check and the error figures (no GPU needed)."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_traffic_record_needs_matching_sources(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    (tmp_path / "profiles").mkdir()
    rec = {"K": {"bytes_per_launch": 123, "sources": ["k.hip"],
                 "sources_sha256": hashlib.sha256(b"kernel v1\n").hexdigest()}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("K") == 123
    assert bench.measured_traffic("other kernel") is None
    src.write_text("kernel v2\n")             # the kernel changed since the counters
    assert bench.measured_traffic("K") is None


def test_committed_traffic_record_is_well_formed():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for key, r in rec.items():
        assert r["bytes_per_launch"] > 0 and r["fetch_scale"] > 0 and r["write_scale"] > 0
        assert all(os.path.exists(os.path.join(ROOT, f)) for f in r["sources"]), key
        assert os.path.exists(os.path.join(ROOT, r["summary"])), key


def test_error_helpers():
    g = np.random.default_rng(3)
    A = g.standard_normal((7, 5)).astype(np.float32)
    B = g.standard_normal((5, 6)).astype(np.float32)
    rows, cols = np.array([0, 3, 6, 6]), np.array([5, 0, 2, 5])
    full = A.astype(np.float64) @ B.astype(np.float64)
    assert np.allclose(bench.ref_sampled(A, B, rows, cols), full[rows, cols], rtol=0, atol=1e-12)
    R = np.array([3.0, 4.0])
    assert bench.relerr(R, R) == 0.0
    assert abs(bench.relerr(np.array([3.0, 4.0 + 0.5]), R) - 0.1) < 1e-15     # ||(0, .5)|| / ||(3, 4)||
    assert bench.relerr(np.array([1.0]), np.array([0.0])) == 1.0             # zero reference: absolute
