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


def test_traffic_dropped_when_kernel_sources_change(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "walk_l64_counters.json")) as f:
        rec = json.load(f)
    monkeypatch.setattr(bench, "kernel_source_sha256", lambda: rec["kernel_source_sha256"])
    gbs = bench.measured_traffic_gbs(0.0634)
    kb = rec["fetch_size_kb_per_launch"] * rec["fetch_scale"] + rec["write_size_kb_per_launch"] * rec["write_scale"]
    assert gbs == pytest.approx(kb * 1024 / 0.0634 / 1e9)
    monkeypatch.setattr(bench, "kernel_source_sha256", lambda: "0" * 64)
    assert bench.measured_traffic_gbs(0.0634) is None


def test_profiled_counters_match_the_current_kernel_sources():
    """The stored counters were taken on the sources in the tree (otherwise
    the benchmark reports no traffic; re-profile after changing them)."""
    with open(os.path.join(ROOT, "profiles", "walk_l64_counters.json")) as f:
        rec = json.load(f)
    assert rec["kernel_source_sha256"] == bench.kernel_source_sha256()
