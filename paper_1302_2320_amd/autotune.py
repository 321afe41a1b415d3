"""Launch autotuner: picks, per lattice side L, the fastest placement of the
walkers' hot state (wl_tuning.placement) and number of walkers per wavefront
(wl_tuning.walkers_per_wave) by timing short windows of a representative
batch on the current GPU.

None of the tuned choices changes a trajectory (the parity tests run every
placement), so the table can be regenerated on any machine without changing
results.  The flatness-check interval does change trajectories and is not
tuned here: it stays a per-line parameter (default 16N).

    python -m paper_1302_2320_amd.autotune [--out PATH] 16 32 64 256   # writes tune_table.json
"""
from __future__ import annotations

import json
import os
import sys
import time

from .workloads import LineSpec

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.json")

# placement codes of wl_tuning.placement
# (placement, walkers per wavefront)
CANDIDATES_SMALL = [(1, 64), (1, 32), (1, 16), (2, 64), (3, 64), (3, 16)]   # L <= 64
CANDIDATES_LARGE = [(0, 64), (0, 32), (0, 16)]                              # L > 64: device memory only


def representative_lines(L: int, walkers: int) -> list:
    """`walkers` walkers spread evenly over the lines 1..N/2 of side L."""
    N = L * L
    half = N // 2
    out = []
    for i in range(walkers):
        ell = 1 + (i * (half - 1)) // max(1, walkers - 1)
        out.append(LineSpec(L=L, ell=ell, seed=1, walker=i % 65536, lnf_min=1e-8))
    return out


def time_candidate(lines, placement: int, wpw: int, attempts: int, steps: int) -> float:
    """Proposals per second of one launch configuration."""
    import torch

    from . import wl

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


def tune(L: int, walkers: int = 16384, attempts: int = 8192, steps: int = 3) -> dict:
    lines = representative_lines(L, walkers)
    cands = CANDIDATES_SMALL if L <= 64 else CANDIDATES_LARGE
    results = []
    for placement, wpw in cands:
        rate = time_candidate(lines, placement, wpw, attempts, steps)
        results.append({"placement": placement, "wpw": wpw, "attempts_per_s": rate})
        print(f"# L={L} placement={placement} wpw={wpw}: {rate:.3e} proposals/s", file=sys.stderr, flush=True)
    best = max(results, key=lambda r: r["attempts_per_s"])
    return {"placement": best["placement"], "wpw": best["wpw"], "candidates": results}


def load_table(path: str = TABLE) -> dict:
    try:
        with open(path) as f:
            return {int(k): v for k, v in json.load(f).items()}
    except OSError:
        return {}


def choice_for(L: int, table: dict | None = None) -> tuple:
    """(placement, walkers per wavefront) for side L: the tuned entry for the
    nearest tuned L, else the library default (0, 0)."""
    table = load_table() if table is None else table
    if not table:
        return 0, 0
    near = min(table, key=lambda x: abs(x - L) + (1000 if (x <= 64) != (L <= 64) else 0))
    e = table[near]
    return int(e["placement"]), int(e["wpw"])


def main(argv):
    import torch
    torch.cuda.set_device(0)
    out = TABLE
    if argv[:1] == ["--out"]:
        out, argv = argv[1], argv[2:]
    Ls = [int(x) for x in argv] or [16, 32, 64]
    table = load_table(out)
    for L in Ls:
        table[L] = tune(L)
    with open(out, "w") as f:
        json.dump({str(k): v for k, v in sorted(table.items())}, f, indent=1)
    print(json.dumps({str(k): {"placement": v["placement"], "wpw": v["wpw"]} for k, v in table.items()}))


if __name__ == "__main__":
    main(sys.argv[1:])
