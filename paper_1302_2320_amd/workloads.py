"""Synthetic workloads: line parameter sets of the benchmark configurations.

Inputs of this method are job descriptors only (lattice side, line, seed,
walker, schedule); every random number a walk uses comes from its own
counter-based stream.  This module holds no part of the method's arithmetic
and is shared by the tests of both the oracle and the GPU library.

Presets (ln f from 1 with f -> f^(1/4), 80% flatness):
  c1      4x4 periodic, all 17 lines, 1 walker, seed 1, ln f_min 1e-6
  c2      8x8 periodic, all 65 lines, seeds 1..4 (walker 0), ln f_min 1e-8
  c3      32x32, lines 0..512, walkers 0..7, seed 1, ln f_min 1e-8
  l64     64x64, lines 0..2048, walkers 0..7, seed 1, ln f_min 1e-8
          (the attempts/s workload at L = 64)
  c5      256x256, lines 0..32768, walker 0, seed 1, ln f_min 1e-8
  job     one served DOS job: lines 0..N/2 of one L, one walker, its seed
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List


@dataclass(frozen=True)
class LineSpec:
    """One walker on one line (the fields of wl_line_params)."""
    L: int
    ell: int
    seed: int = 1
    walker: int = 0
    lnf0: float = 1.0
    lnf_min: float = 1e-8
    flatness: float = 0.8
    check_interval: int = 0
    reset_checks: int = 0     # extra resets at unchanged f (0 = never)
    boundary: int = 0         # 0 periodic, 1 open, 2 periodic with the last row held up
    lattice: int = 0          # 0 square, 1 triangular, 2 honeycomb

    @property
    def nb(self) -> int:
        """Bins of the line: (min(z m, N_B) >> s) + 1 (include/wl.h, Conventions)."""
        L = self.L
        nup = self.ell + (L if self.boundary == 2 else 0)
        m = min(nup, L * L - nup)
        z = {0: 4, 1: 6, 2: 3}[self.lattice]
        o = L * (L - 1)
        op = 1 if self.boundary == 1 else 0
        nbond = {0: (2 * L * L, 2 * o), 1: (3 * L * L, 2 * o + (L - 1) ** 2),
                 2: (3 * L * L // 2, o + o // 2)}[self.lattice][op]
        s = 1 if not op and z % 2 == 0 else 0
        return (min(z * m, nbond) >> s) + 1


def _lines(L, ells, seeds, walkers, lnf_min, flatness=0.8, check_interval=0):
    return [LineSpec(L=L, ell=e, seed=s, walker=w, lnf0=1.0, lnf_min=lnf_min, flatness=flatness,
                       check_interval=check_interval)
            for e in ells for s in seeds for w in walkers]


def c1() -> List[LineSpec]:
    return _lines(4, range(17), [1], [0], 1e-6)


def c2() -> List[LineSpec]:
    return _lines(8, range(65), [1, 2, 3, 4], [0], 1e-8)


def c3(check_interval: int = 0) -> List[LineSpec]:
    return _lines(32, range(513), [1], range(8), 1e-8, check_interval=check_interval)


def l64(walkers: int = 8, check_interval: int = 0) -> List[LineSpec]:
    return _lines(64, range(2049), [1], range(walkers), 1e-8, check_interval=check_interval)


def c5(check_interval: int = 0) -> List[LineSpec]:
    return _lines(256, range(32769), [1], [0], 1e-8, check_interval=check_interval)


def job(L: int, seed: int, lnf_min: float = 1e-7, check_interval: int = 0) -> List[LineSpec]:
    return _lines(L, range(L * L // 2 + 1), [seed], [0], lnf_min, check_interval=check_interval)


def longest_first(lines: List[LineSpec]) -> List[int]:
    """Order (indices) by decreasing line width 2*min(ell, N-ell)+1: the cost of a
    line grows with the number of its bins, so the widest lines start first."""
    return sorted(range(len(lines)), key=lambda i: -lines[i].nb)
