"""Host logic of bench.py (no GPU): the one-GPU refusal, the algorithmic
byte count per proposal, the stored HBM counters written from rocprofv3
output, and the guard that drops the calibrated HBM traffic once the kernel
sources differ from the profiled ones."""
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
    rec = {"kernel": "walk_pc_kernel", "kernel_source_sha256": "a" * 64, "steps": 20, "warmup": 5,
           "launches_per_step": bench.STEP_LAUNCHES,
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
    # the counters belong to one kernel: a run launching another gets none
    assert bench.measured_traffic_gbs(0.05, _args(), str(path), kernel="walk_pc_kernel") == gbs
    assert bench.measured_traffic_gbs(0.05, _args(), str(path), kernel="walk_kernel") is None
    monkeypatch.setattr(bench, "STEP_LAUNCHES", bench.STEP_LAUNCHES + 1)
    assert bench.measured_traffic_gbs(0.05, _args(), str(path)) is None
    monkeypatch.setattr(bench, "STEP_LAUNCHES", rec["launches_per_step"])
    monkeypatch.setattr(bench, "STEP_ATTEMPTS", 1 << 10)
    assert bench.measured_traffic_gbs(0.05, _args(), str(path)) is None
    monkeypatch.setattr(bench, "STEP_ATTEMPTS", rec["attempts_per_launch"])
    monkeypatch.setattr(bench, "kernel_source_sha256", lambda: "0" * 64)
    assert bench.measured_traffic_gbs(0.05, _args(), str(path)) is None


def _counter_csv(folder, rows):
    """A rocprofv3 counter-collection CSV with the columns store_counters reads."""
    folder.mkdir()
    lines = ['"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"']
    lines += [f'{d},"{k}","{c}",{v}' for d, k, c, v in rows]
    (folder / "run_counter_collection.csv").write_text("\n".join(lines) + "\n")


def test_store_counters_averages_the_timed_dispatches(monkeypatch, tmp_path):
    """Per dispatch the counter's rows add up; the stored figure is the mean
    over the dispatches after the warm-up launches; other kernels and other
    counters are ignored; the scale makes the largest dispatch of the copy
    run equal 1 GiB."""
    steps, warmup, kern = 2, 1, "walk_pc_kernel<64, true>"
    n = (steps + warmup) * bench.STEP_LAUNCHES
    w = warmup * bench.STEP_LAUNCHES
    for tag, counter in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        base = 1000.0 if tag == "fetch" else 300.0
        rows = [(0, "init_kernel", counter, 5.0)]
        for d in range(1, n + 1):
            v = 7.0 if d <= w else base + d            # two rows per dispatch: v + 1 and v - 1
            rows += [(d, kern, counter, v + 1), (d, kern, counter, v - 1), (d, kern, "GRBM_COUNT", 9.0)]
        rows += [(n + 1, "stats_kernel", counter, 1e9)]
        _counter_csv(tmp_path / tag, rows)
        copy_kb = (1 << 20) * (1.25 if tag == "fetch" else 0.5)
        _counter_csv(tmp_path / f"copy_{tag}", [(1, "elementwise_kernel", counter, copy_kb),
                                                 (2, "fill_kernel", counter, 12.0)])
    monkeypatch.setattr(bench, "kernel_source_sha256", lambda: "b" * 64)
    out = tmp_path / "counters.json"
    rec = bench.store_counters([str(tmp_path / d) for d in ("fetch", "write", "copy_fetch", "copy_write")],
                               "walk_pc_kernel", steps, warmup, str(out))
    timed = range(w + 1, n + 1)
    assert rec["fetch_size_kb_per_dispatch"] == pytest.approx(sum(2 * (1000.0 + d) for d in timed) / len(timed))
    assert rec["write_size_kb_per_dispatch"] == pytest.approx(sum(2 * (300.0 + d) for d in timed) / len(timed))
    assert rec["dispatches_averaged"] == steps * bench.STEP_LAUNCHES
    assert rec["fetch_scale"] == pytest.approx(0.8) and rec["write_scale"] == pytest.approx(2.0)
    assert json.loads(out.read_text()) == rec
    # the stored record is what the traffic figure reads
    gbs = bench.measured_traffic_gbs(0.05, _args(steps, warmup), str(out))
    assert gbs == pytest.approx((rec["fetch_size_kb_per_dispatch"] * 0.8 + rec["write_size_kb_per_dispatch"] * 2.0)
                                * 1024 / 0.05 / 1e9)
    # a run with another number of launches is refused
    with pytest.raises(ValueError):
        bench.store_counters([str(tmp_path / d) for d in ("fetch", "write", "copy_fetch", "copy_write")],
                             "walk_pc_kernel", steps + 1, warmup, str(out))
