"""Throughput benchmark: Wang-Landau move attempts per second at L = 64.

Workload: the 64x64 periodic lattice, every line ell = 0..2048 (the rest follow
by up-down symmetry) with 8 walkers each (16392 walkers, seed 1, walker
0..7), ln f from 1 towards 1e-8 with f -> f^(1/4), 80% flatness, check
interval 16N.  A step is one launch of the walk kernel that advances every
walker by 65536 proposals (flatness tests and stage transitions included).
Walker state is resident in HBM before timing starts.

Prints one JSON line.  The `roofline` object reports the walk kernel's
algorithmic bytes per second (per-attempt bytes x attempts per launch / mean
launch time from HIP events on the launch stream) against HBM peak;
`cpu_baseline` times the CPU oracle on the host cores over a bounded sample
of the same walkers.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

STEP_ATTEMPTS = 65536
HBM_PEAK_GBS = 8000.0


def bytes_per_attempt(p_acc: float) -> float:
    """Algorithmic bytes one proposal must touch in the walker's state.

    Reads: two list entries (2 x 2 B), the four neighbours of each picked site
    (8 bits of the bit-packed lattice), ln g of the proposed bin (8 B).
    Writes, on acceptance: two list entries (4 B), two spin bits, and ln g
    and h of the bin the walk leaves (16 B)."""
    return 13.0 + p_acc * 20.25


def measured_traffic_gbs(mean_launch_s: float):
    """HBM-side bytes per launch from the stored FETCH_SIZE / WRITE_SIZE
    counters of the walk kernel (scaled by the copy calibration), as GB/s at
    this run's launch time; None when the kernel source has changed since the
    counters were taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "walk_l64_counters.json")
    src = os.path.join(ROOT, "paper_1302_2320_amd", "csrc", "wl_kernels.hip")
    try:
        with open(prof) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    kb = rec["fetch_size_kb_per_launch"] * rec["fetch_scale"] + rec["write_size_kb_per_launch"] * rec["write_scale"]
    return kb * 1024.0 / mean_launch_s / 1e9


def cpu_baseline(lines, target_s: float = 12.0):
    """Oracle attempts/s on the host cores over a bounded sample of the workload."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 64))
    rng = np.random.default_rng(0)
    sample = [lines[int(i)] for i in rng.choice(len(lines), size=cores * 2, replace=False)]
    sample = [p for p in sample if 1 < p.ell < p.L * p.L - 1] or sample
    # calibrate on one walker, then size the per-walker count for ~target_s of wall time
    probe = oracle.Walker(sample[0].L, sample[0].ell, sample[0].seed, sample[0].walker)
    t0 = time.perf_counter()
    probe.advance(200000)
    rate1 = 200000 / (time.perf_counter() - t0)
    per = int(rate1 * target_s * cores / len(sample))

    def run(p):
        w = oracle.Walker(p.L, p.ell, p.seed, p.walker, p.lnf0, p.lnf_min, p.flatness, p.check_interval)
        w.advance(per)
        return w.info().attempts

    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as pool:
        total = sum(pool.map(run, sample))
    el = time.perf_counter() - t0
    return {"value": total / el, "unit": "attempts/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sample)} walkers of the same workload, {per} proposals each from their "
                      f"start state ({total} proposals, {el:.1f} s), one thread per core"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--placement", type=int, default=0,
                    help="hot-state placement for L <= 64 (wl_tuning.placement); 0 = library default")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (scale for HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 1 << 30}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the walkers of a line set are "
                                   "independent, and multi-GPU sharding is not part of this build",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1302_2320_amd import wl, workloads

    torch.cuda.set_device(0)
    lines = workloads.l64()
    print(f"# bench: {len(lines)} walkers (L=64, lines 0..2048 x 8), {STEP_ATTEMPTS} proposals/step, "
          f"warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    batch = wl.Batch(lines, placement=args.placement, stream=stream)
    torch.cuda.synchronize()

    for i in range(args.warmup):
        batch.advance(STEP_ATTEMPTS)
        torch.cuda.synchronize()
        print(f"# warmup step {i} done", file=sys.stderr, flush=True)
    st0 = batch.stats()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        events[i][0].record(stream)
        batch.advance(STEP_ATTEMPTS)
        events[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st1 = batch.stats()
    kern_ms = [a.elapsed_time(b) for a, b in events]
    attempts = int(st1["attempts"].sum() - st0["attempts"].sum())
    accepts = int(st1["accepts"].sum() - st0["accepts"].sum())
    p_acc = accepts / max(attempts, 1)
    value = attempts / wall
    mean_launch_s = (sum(kern_ms) / len(kern_ms)) / 1e3
    per_launch_attempts = attempts / args.steps
    achieved = bytes_per_attempt(p_acc) * per_launch_attempts / mean_launch_s / 1e9
    print(f"# timed {args.steps} steps: {attempts} attempts in {wall:.3f} s, p_acc {p_acc:.3f}, "
          f"launch mean {mean_launch_s * 1e3:.2f} ms", file=sys.stderr, flush=True)

    out = {
        "metric": "WL move attempts/s at L=64",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "64x64 periodic Ising, lines ell=0..2048 x 8 walkers (16392 walkers), "
                               "seed 1, ln f 1 -> 1e-8 (f -> f^1/4), 80% flatness, check interval 16N; "
                               f"one step = {STEP_ATTEMPTS} proposals per walker in one launch",
                   "walkers": len(lines), "attempts_per_step": per_launch_attempts,
                   "acceptance": p_acc},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic_gbs(mean_launch_s) if args.placement == 0 else None,
                     "kernel": "walk_kernel",
                     "bytes_per_attempt": bytes_per_attempt(p_acc),
                     "mean_launch_ms": mean_launch_s * 1e3},
    }
    batch.close()
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(lines)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
