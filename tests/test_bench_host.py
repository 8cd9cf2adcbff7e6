"""bench.py's host-side contract (CPU, no GPU): one GPU only, and the HBM
traffic it reports is read from a committed counter summary only while that
summary's kernel-source hash (and tile shape) match the sources."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_algorithmic_bytes_per_node():
    # PFC sweep: read g 5, f 5, rho^k, omega^k; write g 5 (FP64); 3D: read g 6, f 6, rho^k, omega^k 3; write g 6
    assert bench.SWEEP_BYTES_PFC == 8 * (5 + 5 + 2 + 5) == 136
    assert bench.SWEEP_BYTES_3D == 8 * (6 + 6 + 1 + 3 + 6) == 176
    assert bench.HBM_PEAK_GBS == 8000.0


def test_committed_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    h = bench.source_hash()
    good = tmp_path / "good.md"
    good.write_text(f"x\nsource_hash: {h}\ntile_shape: 64x16x512\ntraffic_bytes_per_launch: 48291406\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(good))
    assert bench.committed_traffic("64x16x512") == 48291406.0
    assert bench.committed_traffic("32x16x512") is None       # another tile shape
    stale = tmp_path / "stale.md"
    stale.write_text("source_hash: 0123456789abcdef\ntile_shape: 64x16x512\ntraffic_bytes_per_launch: 1\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(stale))
    assert bench.committed_traffic("64x16x512") is None       # taken from other sources
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "missing.md"))
    assert bench.committed_traffic("64x16x512") is None


def test_committed_traffic_per_shape_lines(tmp_path, monkeypatch):
    """A summary may carry one traffic line per tile shape
    (traffic_bytes_per_launch_<shape>); each shape reads its own, a shape
    without a line gets None, and a stale hash voids them all."""
    h = bench.source_hash()
    p = tmp_path / "multi.md"
    p.write_text(f"source_hash: {h}\ntraffic_bytes_per_launch_64x16x1024: 38515727\n"
                 "traffic_bytes_per_launch_32x32x1024: 38505275\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(p))
    assert bench.committed_traffic("64x16x1024") == 38515727.0
    assert bench.committed_traffic("32x32x1024") == 38505275.0
    assert bench.committed_traffic("32x16x512") is None
    p.write_text("source_hash: 0123456789abcdef\ntraffic_bytes_per_launch_64x16x1024: 1\n")
    assert bench.committed_traffic("64x16x1024") is None


def test_committed_traffic_3d_follows_the_source_hash(tmp_path, monkeypatch):
    h = bench.source_hash(bench.KERNEL_SOURCES_3D)
    assert h != bench.source_hash()
    p = tmp_path / "p3.md"
    p.write_text(f"source_hash_3d: {h}\ntraffic_bytes_per_sweep_128: 592708325\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY_3D", str(p))
    assert bench.committed_traffic_3d(128) == 592708325.0
    assert bench.committed_traffic_3d(256) is None            # measured at 128^3 only
    p.write_text("source_hash_3d: 0123456789abcdef\ntraffic_bytes_per_sweep_128: 1\n")
    assert bench.committed_traffic_3d(128) is None
