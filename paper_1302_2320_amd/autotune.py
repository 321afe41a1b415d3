"""Launch autotuner.  Per lattice side L it picks, by timing on the current
GPU:

- the placement of the walkers' hot state (wl_tuning.placement) and the
  walkers per wavefront (wl_tuning.walkers_per_wave), from short windows of a
  representative batch; none of these changes a trajectory (the parity tests
  run every placement);
- the flatness-check interval C = factor * N (factor 4, 16 or 64), from the
  time a representative set of narrow lines takes to reach ln f < 1e-2
  (timed for L <= 64; wider lattices keep 16).
  C does change trajectories, so the library applies the tuned factor only to
  lines that ask for it (check_interval = WL_CHECK_INTERVAL_TUNED in
  include/wl.h); the default stays C = 16 N.  Any other implementation of the
  walk reproduces such a line by using C = factor(L) * N from this table.

The lattice layout is not a dimension: the walk keeps the lattice bit-packed
(one 64-bit word per row and walker for L <= 64), which is what lets a row of
neighbours come from one LDS read.

The table (tune_table.json) is compiled into the library by build.py; a
batch created without a wl_tuning takes each launch class's placement and
walkers per wavefront from the entry of its L (the nearest tuned L on the
same side of 64).

    python -m paper_1302_2320_amd.autotune [--out PATH] 8 16 32 64 128 256
"""
from __future__ import annotations

import json
import os
import sys
import time

from .workloads import LineSpec

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.json")

# (placement, walkers per wavefront) of wl_tuning; 0 walkers per wavefront for
# the placements whose kernel fixes it (5 and 8: sixteen, 6 and 7: sixty-four)
CANDIDATES_SMALL = [(1, 64), (1, 32), (1, 16), (2, 64), (3, 64), (3, 16), (5, 0), (6, 0), (7, 0), (8, 0)]   # L <= 64
# L > 64: the lattice in device memory (0) or in LDS (1, sixteen walkers per workgroup)
CANDIDATES_LARGE = [(0, 64), (0, 32), (0, 16), (1, 16)]
CHECK_FACTORS = (4, 16, 64)
DEFAULT_CHECK_FACTOR = 16


def representative_lines(L: int, walkers: int) -> list:
    """`walkers` walkers spread evenly over the lines 1..N/2 of side L."""
    N = L * L
    half = N // 2
    out = []
    for i in range(walkers):
        ell = 1 + (i * (half - 1)) // max(1, walkers - 1)
        out.append(LineSpec(L=L, ell=ell, seed=1, walker=i % 65536, lnf_min=1e-8))
    return out


def narrow_lines(L: int, walkers: int, factor: int, lnf_min: float = 1e-2) -> list:
    """`walkers` walkers on lines 1..max(2, N/16) (lines that end in seconds),
    flatness tested every factor * N proposals."""
    N = L * L
    top = max(2, N // 16)
    return [LineSpec(L=L, ell=1 + (i * (top - 1)) // max(1, walkers - 1), seed=7, walker=i % 65536,
                     lnf_min=lnf_min, check_interval=factor * N) for i in range(walkers)]


def time_candidate(lines, placement: int, wpw: int, attempts: int, steps: int) -> float:
    """Proposals per second of one launch configuration."""
    import torch

    from . import wl

    if lines[0].L > 64:      # wl_tuning.wide_placement for lattices wider than 64
        b = wl.Batch(lines, walkers_per_wave=wpw, wide_placement=3 if placement == 0 else 1)
    else:
        b = wl.Batch(lines, walkers_per_wave=wpw, placement=placement)
    b.advance(attempts)                         # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.advance(attempts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.close()
    return len(lines) * attempts * steps / dt


def time_to_end(lines, limit_s: float) -> dict:
    """Seconds for every walker of `lines` to finish (library launch choices),
    or None past limit_s."""
    import torch

    from . import wl

    t0 = time.perf_counter()
    b = wl.Batch(lines)
    while b.run(1 << 18, 1) > 0:
        if time.perf_counter() - t0 > limit_s:
            b.close()
            return {"seconds": None, "proposals": None}
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = b.stats()
    b.close()
    return {"seconds": dt, "proposals": int(st["attempts"].sum())}


def tune(L: int, walkers: int = 16384, attempts: int = 8192, steps: int = 3, check_walkers: int = 128,
         check_limit_s: float = 40.0) -> dict:
    lines = representative_lines(L, walkers)
    cands = CANDIDATES_SMALL if L <= 64 else CANDIDATES_LARGE
    results = []
    for placement, wpw in cands:
        rate = time_candidate(lines, placement, wpw, attempts, steps)
        results.append({"placement": placement, "wpw": wpw, "attempts_per_s": rate})
        print(f"# L={L} placement={placement} wpw={wpw}: {rate:.3e} proposals/s", file=sys.stderr, flush=True)
    best = max(results, key=lambda r: r["attempts_per_s"])
    checks = []
    for f in (CHECK_FACTORS if L <= 64 else ()):
        r = time_to_end(narrow_lines(L, check_walkers, f), check_limit_s)
        checks.append({"factor": f, **r})
        print(f"# L={L} check interval {f}N: {r['seconds']} s", file=sys.stderr, flush=True)
    done = [c for c in checks if c["seconds"] is not None]
    factor = min(done, key=lambda c: c["seconds"])["factor"] if done else DEFAULT_CHECK_FACTOR
    return {"placement": best["placement"], "wpw": best["wpw"], "check_factor": factor, "candidates": results,
            "check_candidates": checks}


def load_table(path: str = TABLE) -> dict:
    try:
        with open(path) as f:
            return {int(k): v for k, v in json.load(f).items()}
    except OSError:
        return {}


def nearest(L: int, table: dict):
    """The entry of the nearest tuned side on the same side of 64 as L (None if none)."""
    same = [x for x in table if (x <= 64) == (L <= 64)]
    if not same:
        return None
    return table[min(same, key=lambda x: (abs(x - L), x))]


def choice_for(L: int, table: dict | None = None) -> tuple:
    """(placement, walkers per wavefront) for side L; (0, 0), the library
    default, without an entry."""
    table = load_table() if table is None else table
    e = nearest(L, table)
    if e is None:
        return 0, 0
    return int(e["placement"]), int(e["wpw"])


def check_factor_for(L: int, table: dict | None = None) -> int:
    """The tuned flatness-check interval of side L in units of N."""
    table = load_table() if table is None else table
    e = nearest(L, table)
    return int(e.get("check_factor", DEFAULT_CHECK_FACTOR)) if e else DEFAULT_CHECK_FACTOR


def c_header(table: dict) -> str:
    """The table as a C header for the library (one row per tuned L)."""
    rows = []
    for L in sorted(table):
        e = table[L]
        rows.append(f"    {{{L}, {int(e['placement'])}, {int(e['wpw'])}, "
                    f"{int(e.get('check_factor', DEFAULT_CHECK_FACTOR))}}},")
    body = "\n".join(rows) if rows else "    {0, 0, 0, 16},"
    return ("// Generated by build.py from tune_table.json (the launch autotuner's table).\n"
            "#pragma once\n"
            "// L, placement (wl_tuning.placement), walkers per wavefront, check-interval factor\n"
            "static const int kTuneTable[][4] = {\n" + body + "\n};\n"
            f"static const int kTuneTableRows = {len(rows)};\n")


def main(argv):
    import torch
    torch.cuda.set_device(0)
    out = TABLE
    if argv[:1] == ["--out"]:
        out, argv = argv[1], argv[2:]
    Ls = [int(x) for x in argv] or [8, 16, 32, 64, 128, 256]
    table = load_table(out)
    for L in Ls:
        table[L] = tune(L)
        with open(out, "w") as f:
            json.dump({str(k): v for k, v in sorted(table.items())}, f, indent=1)
    print(json.dumps({str(k): {"placement": v["placement"], "wpw": v["wpw"], "check_factor": v["check_factor"]}
                      for k, v in table.items()}))


if __name__ == "__main__":
    main(sys.argv[1:])
