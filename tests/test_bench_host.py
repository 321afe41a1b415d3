"""Host logic of bench.py (no GPU): the one-GPU refusal, the algorithmic
byte count per proposal and the guard that drops the calibrated HBM traffic
once the kernel sources differ from the profiled ones."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]


@pytest.mark.parametrize("lattice", ["square", "triangular", "honeycomb"])
def test_bytes_per_attempt(lattice):
    """Reads: two 2-byte list entries, 2 x degree neighbour bits, one 8-byte
    ln g; writes on acceptance: two list entries, two spin bits, ln g and h
    of the bin left (16 B)."""
    degree = bench.LATTICES[lattice][1]
    assert bench.bytes_per_attempt(0.0, degree) == pytest.approx(4 + 2 * degree / 8 + 8)
    assert bench.bytes_per_attempt(1.0, degree) - bench.bytes_per_attempt(0.0, degree) == pytest.approx(
        4 + 2 / 8 + 16)


def _args(steps=20, warmup=5):
    import argparse
    return argparse.Namespace(steps=steps, warmup=warmup)


def test_traffic_dropped_when_kernel_or_launch_shape_change(monkeypatch, tmp_path):
    rec = {"kernel_source_sha256": "a" * 64, "steps": 20, "warmup": 5, "launches_per_step": bench.STEP_LAUNCHES,
           "attempts_per_launch": bench.STEP_ATTEMPTS,
           "fetch_size_kb_per_dispatch": 1000.0, "write_size_kb_per_dispatch": 500.0,
           "fetch_scale": 2.0, "write_scale": 1.0}
    path = tmp_path / "c.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "kernel_source_sha256", lambda: "a" * 64)
    gbs = bench.measured_traffic_gbs(0.05, _args(), str(path))
    assert gbs == pytest.approx((1000.0 * 2.0 + 500.0) * 1024 / 0.05 / 1e9)
    # per-launch bytes do not depend on how many steps a run times
    assert bench.measured_traffic_gbs(0.05, _args(steps=10, warmup=2), str(path)) == gbs
    monkeypatch.setattr(bench, "STEP_LAUNCHES", bench.STEP_LAUNCHES + 1)
    assert bench.measured_traffic_gbs(0.05, _args(), str(path)) is None
    monkeypatch.setattr(bench, "STEP_LAUNCHES", rec["launches_per_step"])
    monkeypatch.setattr(bench, "STEP_ATTEMPTS", 1 << 10)
    assert bench.measured_traffic_gbs(0.05, _args(), str(path)) is None
    monkeypatch.setattr(bench, "STEP_ATTEMPTS", rec["attempts_per_launch"])
    monkeypatch.setattr(bench, "kernel_source_sha256", lambda: "0" * 64)
    assert bench.measured_traffic_gbs(0.05, _args(), str(path)) is None
