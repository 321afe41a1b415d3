"""Benchmarks of the micromagnetic-ensemble Wang-Landau walk on one GPU.

Default (the headline metric): Wang-Landau move attempts per second at L = 64.
Workload: the 64x64 periodic lattice, every line ell = 0..2048 (the rest follow
by up-down symmetry) with 8 walkers each (16392 walkers, seed 1, walker
0..7), ln f from 1 towards 1e-8 with f -> f^(1/4), 80% flatness, check
interval 16N.  A step is one launch of the walk kernel that advances every
walker by 65536 proposals (flatness tests and stage transitions included).
Walker state is resident in HBM before timing starts.  Prints one JSON line
with a `roofline` object (algorithmic bytes per second of the walk kernel,
from HIP events on the launch stream, against HBM peak, plus the calibrated
HBM traffic of the profiled kernel) and a `cpu_baseline` object (the CPU
oracle on the host cores over a bounded sample of the same walkers).

Other configurations (`--config`), one JSON line each:
  c1    4x4, all 17 lines, seed 1, ln f -> 1e-6: seconds to completion
  c2    8x8, all 65 lines, seeds 1..4, ln f -> 1e-8: seconds to completion
  l64w  the L = 64 workload with --walkers-per-line walkers per line (scaling
        of the rate with the number of walkers in flight)
  c2w   the 8x8 walkers: proposals/s and time per proposal over a window
        (per-walker speed of a placement, e.g. --placement 4)
  c3    32x32, lines 0..512 x 8 walkers: proposals/s over a window
  c3stages  the 32x32 walkers towards --lnf-min for at most --time-limit s:
        per stage, the slowest walker's proposals and when the last walker
        left it (the basis of the time-to-solution estimate)
  c5    256x256, lines 0..32768: proposals/s over a window, HBM footprint
  serve a Poisson stream of whole-DOS jobs through the job server: p50/p99
        latency, lines/s, jobs/h, against one-launch-per-line runs
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

STEP_ATTEMPTS = 65536          # proposals per walker in one launch
STEP_LAUNCHES = 30             # launches in one step of the L = 64 benchmark (20 steps: > 30 s)
HBM_PEAK_GBS = 8000.0


def bytes_per_attempt(p_acc: float, degree: int = 4) -> float:
    """Algorithmic bytes one proposal must touch in the walker's state.

    Reads: two list entries (2 x 2 B), the `degree` neighbours of each picked
    site (2 x degree bits of the bit-packed lattice; 4 on the square
    lattice), ln g of the proposed bin (8 B).
    Writes, on acceptance: two list entries (4 B), two spin bits, and ln g
    and h of the bin the walk leaves (16 B)."""
    return 12.0 + degree / 4.0 + p_acc * 20.25


LATTICES = {"square": (0, 4), "triangular": (1, 6), "honeycomb": (2, 3)}   # code, degree


def kernel_source_sha256() -> str:
    """sha256 over the sources the walk kernels are compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in ("wl_kernels.hip", "wl_device.h", "wl_internal.h"):
        with open(os.path.join(ROOT, "paper_1302_2320_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic_gbs(mean_launch_s: float, args, prof: str | None = None, kernel: str | None = None):
    """HBM-side bytes per launch from the stored FETCH_SIZE / WRITE_SIZE
    counters of the walk kernel (KiB per dispatch, mean over the timed
    dispatches of the profiled benchmark command, scaled by the copy
    calibration), as GB/s at this run's launch time.  None unless the kernel
    sources, the kernel the run launches (when given) and the launch shape
    (proposals per launch, launches per step) are those the counters were
    taken with."""
    prof = prof or os.path.join(ROOT, "profiles", "walk_l64_counters.json")
    try:
        with open(prof) as f:
            rec = json.load(f)
        sha = kernel_source_sha256()
    except OSError:
        return None
    if rec.get("kernel_source_sha256") != sha:
        return None
    if kernel is not None and rec.get("kernel") != kernel:
        return None
    if (rec.get("attempts_per_launch"), rec.get("launches_per_step")) != (STEP_ATTEMPTS, STEP_LAUNCHES):
        return None
    kb = (rec["fetch_size_kb_per_dispatch"] * rec["fetch_scale"] +
          rec["write_size_kb_per_dispatch"] * rec["write_scale"])
    return kb * 1024.0 / mean_launch_s / 1e9


def store_counters(dirs, kernel: str, steps: int, warmup: int, out_path: str) -> dict:
    """Writes the stored HBM counters of the L = 64 walk kernel (read by
    measured_traffic_gbs) from four rocprofv3 --pmc output folders: FETCH_SIZE
    and WRITE_SIZE of the benchmark command with these steps and warm-up
    (each counter in a run of its own), and the same two counters of the
    --copy-calibration run.  Per dispatch the counter's rows are summed; the
    figure kept is the mean over the timed dispatches (those after the
    warm-up launches), and each scale makes the copy's counter equal its
    1 GiB."""
    import csv
    import statistics

    def per_dispatch(folder, counter, sub):
        acc = {}
        with open(os.path.join(folder, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter and sub in r["Kernel_Name"]:
                    k = int(r["Dispatch_Id"])
                    acc[k] = acc.get(k, 0.0) + float(r["Counter_Value"])
        return [acc[k] for k in sorted(acc)]

    fetch_dir, write_dir, copy_fetch_dir, copy_write_dir = dirs
    expect = (steps + warmup) * STEP_LAUNCHES
    kb, copy_kb = {}, {}
    for tag, counter, run_dir, copy_dir in (("fetch", "FETCH_SIZE", fetch_dir, copy_fetch_dir),
                                            ("write", "WRITE_SIZE", write_dir, copy_write_dir)):
        v = per_dispatch(run_dir, counter, kernel)
        if len(v) != expect:
            raise ValueError(f"{run_dir}: {len(v)} dispatches of {kernel} with {counter}, expected {expect}")
        timed = v[warmup * STEP_LAUNCHES:]
        kb[tag] = statistics.mean(timed)
        copies = per_dispatch(copy_dir, counter, "")
        if not copies:
            raise ValueError(f"{copy_dir}: no {counter} rows")
        copy_kb[tag] = max(copies)           # the 1 GiB copy is the largest dispatch of its run
    rec = {"kernel": kernel, "kernel_source_sha256": kernel_source_sha256(), "steps": steps, "warmup": warmup,
           "launches_per_step": STEP_LAUNCHES, "attempts_per_launch": STEP_ATTEMPTS,
           "fetch_size_kb_per_dispatch": kb["fetch"], "write_size_kb_per_dispatch": kb["write"],
           "fetch_scale": round((1 << 30) / 1024 / copy_kb["fetch"], 4),
           "write_scale": round((1 << 30) / 1024 / copy_kb["write"], 4),
           "dispatches_averaged": len(timed),
           "copy_calibration": {"bytes": 1 << 30, "fetch_size_kb": copy_kb["fetch"],
                                "write_size_kb": copy_kb["write"]}}
    with open(out_path, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


# the kernel each wl_tuning.placement runs for L <= 64 on the periodic square lattice
KERNEL_OF_PLACEMENT = {1: "walk_kernel", 2: "walk_kernel", 3: "walk_kernel", 4: "walk_wave_kernel",
                       5: "walk_group_kernel", 6: "walk_pc_kernel", 7: "walk_spec_kernel", 8: "walk_sg_kernel"}


def walk_kernel_name(args, default_shape: bool) -> str:
    """The walk kernel a launch of the L = 64 workload runs: the library's
    choice (the autotuner's table, compiled into the library) unless the
    flags name a placement or the lattice is not the periodic square one."""
    if not default_shape:
        return KERNEL_OF_PLACEMENT.get(args.placement, "walk_kernel") if args.boundary == "periodic" and \
            args.lattice == "square" else "walk_kernel"
    from paper_1302_2320_amd import autotune
    placement, _ = autotune.choice_for(64)
    return KERNEL_OF_PLACEMENT.get(placement, "walk_kernel")


def host_cores() -> int:
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return max(1, min(cores, 64))


def cpu_baseline(lines, target_s: float = 12.0, sample_size: int | None = None):
    """Oracle proposals/s on the host cores over a bounded sample of the workload."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle

    cores = host_cores()
    rng = np.random.default_rng(0)
    cand = [p for p in lines if 1 < p.ell < p.L * p.L - 1] or lines
    k = min(len(cand), sample_size or cores * 2)
    sample = [cand[int(i)] for i in rng.choice(len(cand), size=k, replace=False)]
    # calibrate on one walker, then size the per-walker count for ~target_s of wall time
    probe = oracle.Walker(sample[0].L, sample[0].ell, sample[0].seed, sample[0].walker,
                          boundary=sample[0].boundary, lattice=sample[0].lattice)
    t0 = time.perf_counter()
    probe.advance(200000)
    rate1 = 200000 / (time.perf_counter() - t0)
    per = max(1, int(rate1 * target_s * min(cores, len(sample)) / len(sample)))

    def run(p):
        w = oracle.Walker(p.L, p.ell, p.seed, p.walker, p.lnf0, p.lnf_min, p.flatness, p.check_interval,
                          reset_checks=p.reset_checks, boundary=p.boundary, lattice=p.lattice)
        w.advance(per)
        return w.info().attempts

    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as pool:
        total = sum(pool.map(run, sample))
    el = time.perf_counter() - t0
    return {"value": total / el, "unit": "attempts/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sample)} walkers of the same workload, up to {per} proposals each from their "
                      f"start state ({total} proposals, {el:.1f} s), one thread per core"}


def timed_window(batch, steps, warmup, attempts_per_launch, stream, launches=1):
    """`warmup` then `steps` steps of `launches` advances each; returns
    (attempts, accepts, wall_s, launch_ms list, warm-up attempts, warm-up s).
    Launch times come from HIP events recorded on the launch stream."""
    import torch
    stw = batch.stats()
    tw = time.perf_counter()
    for i in range(warmup):
        for _ in range(launches):
            batch.advance(attempts_per_launch)
        torch.cuda.synchronize()
        print(f"# warmup step {i} done", file=sys.stderr, flush=True)
    warm_s = time.perf_counter() - tw
    st0 = batch.stats()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps * launches)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        for j in range(launches):
            ev = events[i * launches + j]
            ev[0].record(stream)
            batch.advance(attempts_per_launch)
            ev[1].record(stream)
        if launches > 1:
            torch.cuda.synchronize()
            print(f"# step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st1 = batch.stats()
    kern_ms = [a.elapsed_time(b) for a, b in events]
    attempts = int(st1["attempts"].sum() - st0["attempts"].sum())
    accepts = int(st1["accepts"].sum() - st0["accepts"].sum())
    warm_attempts = int(st0["attempts"].sum() - stw["attempts"].sum())
    return attempts, accepts, wall, kern_ms, warm_attempts, warm_s


def with_boundary(args, lines, name):
    """The workload's lines on the boundary (`--boundary`) and lattice
    (`--lattice`) asked for."""
    if args.boundary == "open":
        lines = [dataclasses.replace(p, boundary=1) for p in lines]
        name = name.replace("periodic", "open")
    code, _ = LATTICES[args.lattice]
    if code:
        lines = [dataclasses.replace(p, lattice=code) for p in lines]
        name = (name.replace("Ising", f"{args.lattice} Ising") if "Ising" in name
                else f"{name}, {args.lattice} lattice")
    return lines, name


def bench_l64(args):
    import torch

    from paper_1302_2320_amd import wl, workloads

    lines, wname = with_boundary(args, workloads.l64(),
                                 "64x64 periodic Ising, lines ell=0..2048 x 8 walkers (16392 walkers), ")
    print(f"# bench: {len(lines)} walkers (L=64, lines 0..2048 x 8), {STEP_LAUNCHES} launches of "
          f"{STEP_ATTEMPTS} proposals per step, warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    batch = wl.Batch(lines, placement=args.placement, walkers_per_wave=args.wpw, stream=stream)
    torch.cuda.synchronize()
    attempts, accepts, wall, kern_ms, warm_att, warm_s = timed_window(batch, args.steps, args.warmup,
                                                                      STEP_ATTEMPTS, stream, STEP_LAUNCHES)
    p_acc = accepts / max(attempts, 1)
    value = attempts / wall
    mean_launch_s = (sum(kern_ms) / len(kern_ms)) / 1e3
    per_launch_attempts = attempts / (args.steps * STEP_LAUNCHES)
    degree = LATTICES[args.lattice][1]
    achieved = bytes_per_attempt(p_acc, degree) * per_launch_attempts / mean_launch_s / 1e9
    print(f"# timed {args.steps} steps: {attempts} attempts in {wall:.3f} s, p_acc {p_acc:.3f}, "
          f"launch mean {mean_launch_s * 1e3:.2f} ms", file=sys.stderr, flush=True)
    default_shape = (args.placement == 0 and args.wpw == 0 and args.boundary == "periodic"
                     and args.lattice == "square")
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
        "config": {"workload": wname +
                               "seed 1, ln f 1 -> 1e-8 (f -> f^1/4), 80% flatness, check interval 16N; "
                               f"one step = {STEP_LAUNCHES} launches of {STEP_ATTEMPTS} proposals per walker",
                   "walkers": len(lines), "attempts_per_step": attempts / args.steps,
                   "acceptance": p_acc,
                   "whole_run": {"attempts": attempts + warm_att, "seconds": wall + warm_s,
                                 "attempts_per_s": (attempts + warm_att) / (wall + warm_s),
                                 "warmup_s": warm_s}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (measured_traffic_gbs(mean_launch_s, args, kernel=walk_kernel_name(args, True))
                                 if default_shape else None),
                     "kernel": walk_kernel_name(args, default_shape),
                     "bytes_per_attempt": bytes_per_attempt(p_acc, degree),
                     "attempts_per_launch": per_launch_attempts,
                     "mean_launch_ms": mean_launch_s * 1e3},
    }
    batch.close()
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(lines)
    print(json.dumps(out), flush=True)


def bench_to_completion(args, name, lines, chunk):
    """Runs every walker of `lines` to ln f < ln f_min; reports seconds."""
    import numpy as np
    import torch

    from paper_1302_2320_amd import wl

    lines, name = with_boundary(args, lines, name)
    if args.reset_checks:
        lines = [dataclasses.replace(p, reset_checks=args.reset_checks) for p in lines]
        name += f", extra resets after {args.reset_checks} non-flat tests"
    if args.check_interval:
        lines = [dataclasses.replace(p, check_interval=args.check_interval) for p in lines]
        name += f", flatness tested every {args.check_interval} proposals"
    if args.half_lines:
        N = lines[0].L * lines[0].L
        lines = [p for p in lines if p.ell <= N // 2]
        name = name.replace("all 65 lines", "lines 0..32 (the rest by symmetry)")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch = wl.Batch(lines, placement=args.placement, walkers_per_wave=args.wpw, stream=stream,
                     tail_walkers=args.tail_walkers)
    last = t0
    while True:
        active = batch.run(chunk, 1)            # one chunk, then the count (synchronises)
        now = time.perf_counter()
        if now - last > 10.0:
            print(f"# {now - t0:.0f} s: {active} walkers active", file=sys.stderr, flush=True)
            last = now
        if active == 0:
            break
    wall = time.perf_counter() - t0
    st = batch.stats()
    attempts = st["attempts"].astype(np.int64)
    out = {"metric": f"seconds to ln f < ln f_min, {name}", "value": wall, "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": name, "walkers": len(lines), "chunk": chunk,
                      "tail_walkers": args.tail_walkers, "reset_checks": args.reset_checks,
                      "check_interval": args.check_interval or "16N"},
           "attempts_total": int(attempts.sum()), "attempts_max_walker": int(attempts.max()),
           "attempts_per_s": float(attempts.sum() / wall),
           "all_done": bool((st["done"] == 1).all())}
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(lines, sample_size=min(len(lines), host_cores()))
    batch.close()
    print(json.dumps(out), flush=True)


def bench_stages(args, name, lines, chunk):
    """Runs `lines` towards ln f < --lnf-min for at most --time-limit seconds
    and records, per stage (ln f = 4^-s), the proposals of the walker that
    spent the most on it and the wall time at which the last walker left it
    (sampled once per launch of `chunk` proposals, so stages shorter than a
    launch are merged into the launch that ends them)."""
    import numpy as np
    import torch

    from paper_1302_2320_amd import wl

    lines = [dataclasses.replace(p, lnf_min=args.lnf_min) for p in lines]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch = wl.Batch(lines, placement=args.placement, walkers_per_wave=args.wpw, stream=stream,
                     tail_walkers=args.tail_walkers)
    n = len(lines)
    prev_stage = np.zeros(n, dtype=np.int64)
    stage_begin = np.zeros(n, dtype=np.int64)       # attempts at which each walker entered its stage
    spent = {}                                      # stage -> max proposals over walkers
    left_at = {}                                    # stage -> wall time the last walker left it
    last = t0
    while True:
        active = batch.run(chunk, 1)
        now = time.perf_counter()
        st = batch.stats()
        att = st["attempts"].astype(np.int64)
        stg = st["stages"].astype(np.int64)
        for i in np.nonzero(stg > prev_stage)[0]:
            s = int(prev_stage[i])
            spent[s] = max(spent.get(s, 0), int(att[i] - stage_begin[i]))
            for s2 in range(s, int(stg[i])):
                left_at[s2] = now - t0
            stage_begin[i] = att[i]
            prev_stage[i] = stg[i]
        if now - last > 10.0:
            print(f"# {now - t0:.0f} s: {active} walkers active, lowest stage {int(stg.min())}",
                  file=sys.stderr, flush=True)
            last = now
        if active == 0 or now - t0 > args.time_limit:
            break
    wall = time.perf_counter() - t0
    batch.close()
    out = {"metric": f"stage profile, {name}", "value": wall, "unit": "s", "higher_is_better": False,
           "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": name + f", ln f_min {args.lnf_min}", "walkers": n, "chunk": chunk,
                      "time_limit_s": args.time_limit},
           "finished": bool(active == 0), "walkers_active": int(active),
           "attempts_total": int(att.sum()), "attempts_max_walker": int(att.max()),
           "stages": [{"stage": s, "lnf": 4.0 ** -s, "max_walker_proposals": spent[s],
                       "all_left_s": left_at.get(s)} for s in sorted(spent)]}
    print(json.dumps(out), flush=True)


def bench_slow_walker(args):
    """ns per proposal of the walker that sets C2's time to solution (8x8,
    ell = 48, seed 3) alone on the device, late in its run: advanced
    `--pre` proposals first (untimed), then `--steps` launches of 2^22."""
    import torch

    from paper_1302_2320_amd import wl, workloads

    p = [x for x in workloads.c2() if x.ell == 48 and x.seed == 3][0]
    stream = torch.cuda.current_stream()
    batch = wl.Batch([p], placement=args.placement or 4, walkers_per_wave=args.wpw, stream=stream)
    chunk = 1 << 22
    for _ in range(args.pre // chunk):
        batch.advance(chunk)
    torch.cuda.synchronize()
    s0 = batch.read_walker(0).stats
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        batch.advance(chunk)
    ev1.record(stream)
    torch.cuda.synchronize()
    s1 = batch.read_walker(0).stats
    n = s1["attempts"] - s0["attempts"]
    ms = ev0.elapsed_time(ev1)
    out = {"metric": "ns per proposal, slowest C2 walker (8x8, ell 48, seed 3), late stage", "value": ms * 1e6 / n,
           "unit": "ns", "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "8x8 periodic, ell 48, seed 3, ln f 1 -> 1e-8", "pre": args.pre,
                      "proposals": int(n), "placement": args.placement or 4},
           "stage": int(s1["stages"]), "acceptance": (s1["accepts"] - s0["accepts"]) / max(n, 1)}
    batch.close()
    print(json.dumps(out), flush=True)


def bench_thermo(args):
    """wl_thermo on a 64x64 plane ((N+1)^2 = 16.8M bins, 134 MB) at 256
    (beta, H) points: points per second and the FP64 exponentials per second
    it sustains (one per supported bin per point)."""
    import numpy as np
    import torch

    from paper_1302_2320_amd import wl

    L = 64
    N = L * L
    rng = np.random.default_rng(5)
    ell = np.arange(N + 1)[:, None]
    q = np.arange(N + 1)[None, :]
    m = np.minimum(ell, N - ell)
    lng = np.where(q <= 2 * m, 0.5 * N * (1.0 - ((q - m) / (m + 1.0)) ** 2), -np.inf)
    lng = lng + np.where(np.isfinite(lng), rng.normal(0.0, 0.5, lng.shape), 0.0)
    support = int(np.isfinite(lng).sum())
    dev = torch.from_numpy(np.ascontiguousarray(lng)).cuda()
    n = 256
    beta = torch.linspace(0.1, 1.0, n, dtype=torch.float64)
    H = torch.linspace(-0.5, 0.5, n, dtype=torch.float64)
    for _ in range(args.warmup):
        wl.thermo(L, dev, beta, H, 1.0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        wl.thermo(L, dev, beta, H, 1.0)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    out = {"metric": "thermodynamic points per second, 64x64 plane", "value": n / (ms * 1e-3), "unit": "points/s",
           "higher_is_better": True, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "64x64 ln g(k, ell) plane, 256 (beta, H) points", "bins": (N + 1) ** 2,
                      "supported_bins": support},
           "ms_per_call": ms, "exp_per_s": support * n / (ms * 1e-3),
           "plane_reads_gb_per_s": (N + 1) ** 2 * 8 * 2 * (n // 4) / (ms * 1e-3) / 1e9}
    print(json.dumps(out), flush=True)


def bench_window(args, name, lines, step_attempts):
    """Proposals/s of a large line set over a window of `args.steps` launches."""
    import torch

    from paper_1302_2320_amd import wl

    lines, name = with_boundary(args, lines, name)

    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    batch = wl.Batch(lines, placement=args.placement, walkers_per_wave=args.wpw, stream=stream)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    attempts, accepts, wall, kern_ms, _, _ = timed_window(batch, args.steps, args.warmup, step_attempts, stream)
    out = {"metric": f"WL move attempts/s, {name}", "value": attempts / wall, "unit": "attempts/s",
           "higher_is_better": True, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "steps": args.steps, "warmup": args.warmup,
           "config": {"workload": name, "walkers": len(lines), "attempts_per_step": step_attempts,
                      "placement": args.placement, "walkers_per_wave": args.wpw},
           "acceptance": accepts / max(attempts, 1), "mean_launch_ms": sum(kern_ms) / len(kern_ms),
           "ns_per_proposal_step": sum(kern_ms) / len(kern_ms) * 1e6 / step_attempts,
           "workspace_gb": batch.ws_bytes / 1e9, "init_s": t_init}
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(lines)
    batch.close()
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """A Poisson stream of whole-DOS jobs through the job server.

    Jobs: L drawn uniformly from --serve-L, one walker per line, lines
    0..N/2, job i seeded 1000 + i, ln f 1 -> --serve-lnf-min.  Capacity is
    the jobs/s of the server when a calibration set of jobs of the same mix is
    submitted at once; the stream then arrives at rho x capacity.  Latency is
    arrival to assembled result (server timestamps).  Baseline (the same kind
    of work as plain one-launch-per-line runs): lines drawn uniformly from
    the stream's jobs are run one at a time with wl_line_run for a fixed time
    budget; its lines/s over the mean lines per job gives its jobs/h."""
    import threading

    import numpy as np

    from paper_1302_2320_amd import wl

    L_set = [int(x) for x in args.serve_L.split(",")]
    lnf_min = args.serve_lnf_min
    rng = np.random.default_rng(20260101)
    MiB = 1 << 20

    def job_L(n):
        return [int(L_set[i]) for i in rng.integers(0, len(L_set), n)]

    # capacity: all calibration jobs at once (or given, to profile the stream alone)
    calib = job_L(args.serve_calib)
    srv = wl.Server(args.serve_budget_mb * MiB)
    if args.serve_capacity > 0:
        capacity = args.serve_capacity
    else:
        t0 = time.perf_counter()
        ids = [srv.submit(L=L, W=1, seed=1000 + i, lnf_min=lnf_min) for i, L in enumerate(calib)]
        for n_done, j in enumerate(ids):
            srv.wait(j, 3600.0)
            print(f"# calibration: {n_done + 1}/{len(ids)} jobs done, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
        cap_wall = time.perf_counter() - t0
        for j in ids:
            srv.fetch(j)
        capacity = len(calib) / cap_wall
        print(f"# capacity {capacity:.3f} jobs/s ({len(calib)} jobs in {cap_wall:.1f} s)", file=sys.stderr,
              flush=True)

    rho = args.serve_rho
    Ls = job_L(args.serve_jobs)
    gaps = rng.exponential(1.0 / (rho * capacity), size=len(Ls))
    sub = []

    def producer():
        for i, (L, g) in enumerate(zip(Ls, gaps)):
            time.sleep(g)
            sub.append(srv.submit(L=L, W=1, seed=5000 + i, lnf_min=lnf_min))

    t0 = time.perf_counter()
    win0 = time.monotonic_ns()         # the stream's window on the clock of kernel traces
    th = threading.Thread(target=producer)
    th.start()
    while th.is_alive():
        th.join(10.0)
        print(f"# stream: {len(sub)}/{len(Ls)} jobs submitted, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    last = time.perf_counter()
    for n_done, j in enumerate(sub):
        srv.wait(j, 3600.0)
        if time.perf_counter() - last > 10.0:
            print(f"# stream: {n_done + 1}/{len(sub)} jobs done, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
            last = time.perf_counter()
    wall = time.perf_counter() - t0
    win1 = time.monotonic_ns()
    lat = []
    for j in sub:
        st = srv.job_stats(j)
        lat.append(st["done_s"] - st["submit_s"])
        srv.fetch(j)
    srv.close()
    lat = np.array(lat)
    n_lines = sum(L * L // 2 + 1 for L in Ls)
    served = {"jobs": len(Ls), "rho": rho, "p50_s": float(np.percentile(lat, 50)),
              "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
              "lines_per_s": n_lines / wall, "jobs_per_h": len(Ls) / wall * 3600.0, "wall_s": wall,
              "window_monotonic_ns": [win0, win1]}
    print(f"# rho {rho}: p50 {served['p50_s']:.2f} s p99 {served['p99_s']:.2f} s, "
          f"{served['jobs_per_h']:.0f} jobs/h", file=sys.stderr, flush=True)

    # baseline: lines drawn uniformly from the stream's jobs, one wl_line_run each
    pool = [(L, ell, 5000 + i) for i, L in enumerate(Ls) for ell in range(L * L // 2 + 1)]
    order = rng.permutation(len(pool)) if args.serve_baseline_s > 0 else []
    t0 = time.perf_counter()
    done_lines, proposals = 0, 0
    for idx in order:
        L, ell, seed = pool[int(idx)]
        _, st = wl.line_run(L, ell, seed, 1.0, lnf_min, 0.8)
        done_lines += 1
        proposals += st["attempts"]
        if time.perf_counter() - t0 > args.serve_baseline_s:
            break
    base_wall = time.perf_counter() - t0
    mean_lines = n_lines / len(Ls)
    base_lines_per_s = done_lines / base_wall if done_lines else None
    out = {"metric": "served DOS jobs: p50/p99 latency", "value": served["p50_s"], "unit": "s",
           "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"Poisson stream of {len(Ls)} whole-DOS jobs at rho {rho}, L uniform in "
                                  f"{L_set}, one walker per line, lines 0..N/2, ln f 1 -> {lnf_min}, "
                                  "80% flatness, seeds 5000+i",
                      "budget_mb": args.serve_budget_mb, "lnf_min": lnf_min},
           "p99_s": served["p99_s"], "capacity_jobs_per_s": capacity, "mean_lines_per_job": mean_lines,
           "served": served,
           "plain_per_line": {"lines_run": done_lines, "seconds": base_wall, "proposals": int(proposals),
                              "lines_per_s": base_lines_per_s,
                              "jobs_per_h": base_lines_per_s / mean_lines * 3600.0 if done_lines else None,
                              "method": "lines drawn uniformly from the stream's jobs, one wl_line_run "
                                        "(one walker, its own launches) each, for a fixed time budget"}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--serve-L", default="16,24,32,48,64")
    ap.add_argument("--serve-lnf-min", type=float, default=0.3,
                    help="serve: ln f_min of every job (0.3: one stage of ln f = 1)")
    ap.add_argument("--serve-jobs", type=int, default=200)
    ap.add_argument("--serve-calib", type=int, default=40)
    ap.add_argument("--serve-rho", type=float, default=0.8)
    ap.add_argument("--serve-capacity", type=float, default=0.0,
                    help="serve: capacity in jobs/s instead of calibrating it (0: calibrate)")
    ap.add_argument("--serve-baseline-s", type=float, default=120.0,
                    help="serve: seconds of one-launch-per-line baseline runs")
    ap.add_argument("--serve-budget-mb", type=int, default=16384)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="l64",
                    choices=["l64", "l64w", "c1", "c2", "c2w", "c2slow", "c3", "c3stages", "c5", "serve", "thermo"])
    ap.add_argument("--check-interval", type=int, default=0,
                    help="c1/c2: proposals between flatness tests (0: the default 16N)")
    ap.add_argument("--half-lines", action="store_true",
                    help="c1/c2: only the lines ell <= N/2 (the rest follow by symmetry)")
    ap.add_argument("--lattice", default="square", choices=list(LATTICES),
                    help="l64: lattice of the walkers (square is the paper's)")
    ap.add_argument("--boundary", default="periodic", choices=["periodic", "open"],
                    help="lattice boundary of the l64 / c1 / c2 / window workloads")
    ap.add_argument("--pre", type=int, default=100_000_000,
                    help="c2slow: proposals run before the timed window")
    ap.add_argument("--walkers-per-line", type=int, default=8, help="l64w: walkers per line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuned", action="store_true",
                    help="take placement and walkers per wavefront from paper_1302_2320_amd/tune_table.json")
    ap.add_argument("--tail-walkers", type=int, default=0,
                    help="run-to-end switch to one wavefront per walker (wl_tuning.tail_walkers); "
                         "0 = library default, -1 = never")
    ap.add_argument("--wpw", type=int, default=0,
                    help="walkers per wavefront (wl_tuning.walkers_per_wave: 16, 32, 64); 0 = library default")
    ap.add_argument("--placement", type=int, default=0,
                    help="hot-state placement for L <= 64 (wl_tuning.placement); 0 = library default")
    ap.add_argument("--reset-checks", type=int, default=0,
                    help="c1/c2: extra histogram resets at unchanged f after this many non-flat tests "
                         "(0 = the plain schedule)")
    ap.add_argument("--lnf-min", type=float, default=1e-3, help="c3stages: ln f_min of the stage profile")
    ap.add_argument("--time-limit", type=float, default=600.0, help="c3stages: seconds before the profile stops")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (scale for HBM byte counters) and exit")
    ap.add_argument("--store-counters", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="host only: write profiles/walk_l64_counters.json from the rocprofv3 --pmc folders of "
                         "the benchmark command (its --steps / --warmup) and of --copy-calibration, and exit")
    args = ap.parse_args()
    if args.store_counters:
        rec = store_counters(args.store_counters, walk_kernel_name(args, True), args.steps, args.warmup,
                             os.path.join(ROOT, "profiles", "walk_l64_counters.json"))
        print(json.dumps(rec))
        return
    if args.tuned:
        # placement and walkers per wavefront from the autotuner's table for
        # the workload's lattice side (explicit flags are overridden)
        from paper_1302_2320_amd import autotune
        side = {"l64": 64, "l64w": 64, "c1": 4, "c2": 8, "c2w": 8, "c2slow": 8, "c3": 32, "c3stages": 32, "c5": 256,
                "serve": 16, "thermo": 64}[args.config]
        args.placement, args.wpw = autotune.choice_for(side)
        print(f"# tuned for L={side}: placement {args.placement}, walkers per wavefront {args.wpw}",
              file=sys.stderr, flush=True)
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
                                   "independent, and sharding them across GPUs is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1302_2320_amd import workloads

    torch.cuda.set_device(0)
    if args.config == "l64":
        bench_l64(args)
    elif args.config == "c1":
        bench_to_completion(args, "4x4 periodic, all 17 lines, seed 1, ln f 1 -> 1e-6", workloads.c1(), 1 << 16)
    elif args.config == "c2":
        bench_to_completion(args, "8x8 periodic, all 65 lines, seeds 1..4, ln f 1 -> 1e-8", workloads.c2(), 1 << 21)
    elif args.config == "c3stages":
        bench_stages(args, "32x32 periodic, lines 0..512 x 8 walkers, seed 1", workloads.c3(), 1 << 21)
    elif args.config == "l64w":
        W = args.walkers_per_line
        bench_window(args, f"64x64 periodic, lines 0..2048 x {W} walkers, seed 1, ln f 1 -> 1e-8",
                     workloads.l64(W), STEP_ATTEMPTS)
    elif args.config == "c2w":
        bench_window(args, "8x8 periodic, all 65 lines, seeds 1..4, ln f 1 -> 1e-8", workloads.c2(), 64 * 1024)
    elif args.config == "c2slow":
        bench_slow_walker(args)
    elif args.config == "thermo":
        bench_thermo(args)
    elif args.config == "c3":
        bench_window(args, "32x32 periodic, lines 0..512 x 8 walkers, seed 1, ln f 1 -> 1e-8",
                     workloads.c3(), 16 * 1024)
    elif args.config == "c5":
        bench_window(args, "256x256 periodic, lines 0..32768, seed 1, ln f 1 -> 1e-8", workloads.c5(), 16 * 1024)
    elif args.config == "serve":
        bench_serve(args)


if __name__ == "__main__":
    main()
