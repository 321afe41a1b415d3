"""Pins of the CPU oracle against what the paper and the mathematics fix.

Known-answer vectors for the generator, libm for the exponential,
hand-worked flatness cases, a full recount of k after every accepted move,
list/lattice consistency, the stage schedule f -> f^(1/4), ergodicity (the
visited bins equal the exact support), and the assembled DOS against the
brute-force enumeration of the 4x4 torus.
"""
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from oracle import exact

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                w = [int(x, 16) for x in line.split()]
                rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert [int(x) for x in oracle.philox4x32_10(ctr, key)] == out


def test_philox_index_draw_uniform():
    # floor(r * n / 2^32) over consecutive counters: chi-square of 8 cells
    n, cells, draws = 1000, 8, 20000
    counts = np.zeros(cells)
    for t in range(draws):
        r = oracle.philox4x32_10([t, 0, 7, 3], [1, 0])
        a = (int(r[0]) * n) >> 32
        counts[a * cells // n] += 1
    exp_ = draws / cells
    chi2 = float(((counts - exp_) ** 2 / exp_).sum())
    assert chi2 < 24.3      # p = 0.001 for 7 degrees of freedom


def test_exp_fixed_against_libm():
    rng = np.random.default_rng(12345)
    xs = np.concatenate([-rng.random(20000) * 700.0, -rng.random(20000) * 2.0,
                         -rng.random(2000) * 1e-8, np.array([-0.0, 0.0, -700.0, -1e-300, -0.5 * math.log(2)])])
    worst = 0.0
    for x in xs:
        got, ref = oracle.exp_fixed(float(x)), math.exp(float(x))
        worst = max(worst, abs(got - ref) / ref)
    assert worst <= 4e-16
    assert oracle.exp_fixed(0.0) == 1.0 and oracle.exp_fixed(-0.0) == 1.0
    assert oracle.exp_fixed(-700.0000001) == 0.0 and oracle.exp_fixed(-1e4) == 0.0


def test_exp_fixed_monotone_near_grid():
    # across the rounding boundaries of n = rint(x / ln 2)
    xs = np.sort(-np.concatenate([np.arange(1, 60) * math.log(2) + d for d in (-1e-12, 0.0, 1e-12)]))
    vals = [oracle.exp_fixed(float(x)) for x in xs]
    assert all(a <= b for a, b in zip(vals, vals[1:]))


def test_flatness_hand_cases():
    # 5 visited bins, S = 40, mean 8, threshold 6.4: four bins pass, 4 >= 0.8*5
    assert oracle.histogram_flat([10, 10, 10, 10, 0], [1] * 5, 0.8, 5) == (True, 5)
    # three pass: 3 < 4
    assert oracle.histogram_flat([10, 10, 10, 0, 0], [1] * 5, 0.8, 5) == (False, 5)
    # a new bin since the previous test blocks flatness
    assert oracle.histogram_flat([10, 10, 10, 10, 0], [1] * 5, 0.8, 4) == (False, 5)
    # unvisited bins do not count: n = 4
    assert oracle.histogram_flat([7, 7, 0, 7, 7], [1, 1, 0, 1, 1], 0.8, 4) == (True, 4)
    # S = 80, threshold h*5 >= 64: 20, 20, 20, 15 pass (4 >= 4)
    assert oracle.histogram_flat([20, 20, 20, 15, 5], [1] * 5, 0.8, 5) == (True, 5)
    # 12*5 = 60 < 64: only three pass
    assert oracle.histogram_flat([20, 20, 20, 12, 8], [1] * 5, 0.8, 5) == (False, 5)
    # exactly at the threshold counts (>=): S = 100, 16*5 = 80 = 0.8*100
    assert oracle.histogram_flat([16, 16, 21, 21, 26], [1] * 5, 0.8, 5) == (True, 5)
    assert oracle.histogram_flat([15, 15, 22, 22, 26], [1] * 5, 0.8, 5) == (False, 5)


@pytest.mark.parametrize("L,ell", [(4, 1), (4, 5), (4, 8), (4, 13), (6, 9), (6, 18), (8, 7), (8, 32), (8, 60)])
def test_walk_recount_and_consistency(L, ell):
    N = L * L
    w = oracle.Walker(L, ell, seed=99, walker=3, lnf_min=1e-4, check_interval=64 * N, debug=True)
    for _ in range(20):
        w.advance(5000)                  # raises if the debug recount disagrees
        s = w.state()
        assert s.k == oracle.count_k(L, s.spins)
        assert sorted(s.up.tolist()) == np.flatnonzero(s.spins == 1).tolist()
        assert sorted(s.dn.tolist()) == np.flatnonzero(s.spins == 0).tolist()
        assert s.k % 2 == 0 and 0 <= s.k <= 4 * min(ell, N - ell)
        if s.done:
            break


def test_edge_lines():
    for L in (4, 8):
        N = L * L
        for ell in (0, N):
            lng, info = oracle.line_run(L, ell, seed=1)
            assert lng.tolist() == [0.0] and info.attempts == 0 and info.done == 1
        for ell in (1, N - 1):
            lng, info = oracle.line_run(L, ell, seed=1)
            # only k = 4 is reachable; flat at the first test, one test per stage
            assert np.isinf(lng[0]) and np.isinf(lng[1]) and lng[2] == 0.0
            assert info.stages == 10 and info.attempts == 10 * 16 * N


def test_stage_schedule():
    lng, info = oracle.line_run(4, 6, seed=5, lnf0=1.0, lnf_min=1e-8)
    assert info.stages == 14 and info.lnf == 4.0 ** -14
    lng, info = oracle.line_run(4, 6, seed=5, lnf0=1.0, lnf_min=1e-6)
    assert info.stages == 10 and info.lnf == 4.0 ** -10


def test_deterministic_and_stream_separation():
    a, ia = oracle.line_run(4, 7, seed=11)
    b, ib = oracle.line_run(4, 7, seed=11)
    assert np.array_equal(a, b) and ia.attempts == ib.attempts
    c, ic = oracle.line_run(4, 7, seed=11, walker=1)
    d, idd = oracle.line_run(4, 7, seed=12)
    assert not np.array_equal(a, c) and not np.array_equal(a, d)


def test_invalid_parameters():
    for kw in (dict(L=5, ell=1), dict(L=2, ell=1), dict(L=258, ell=1), dict(L=4, ell=17),
               dict(L=4, ell=-1), dict(L=4, ell=3, lnf0=1e-9), dict(L=4, ell=3, flatness=0.0),
               dict(L=4, ell=3, flatness=1.5), dict(L=4, ell=3, lnf_min=0.0)):
        with pytest.raises(ValueError):
            oracle.line_run(seed=1, **kw)


def _run_lines(L, seeds, lnf_min, C):
    N = L * L
    jobs = [(ell, s) for ell in range(N + 1) for s in seeds]
    with ThreadPoolExecutor(8) as pool:
        res = list(pool.map(lambda j: oracle.line_run(L, j[0], j[1], lnf_min=lnf_min, check_interval=C), jobs))
    W = len(seeds)
    return [np.stack([res[ell * W + i][0] for i in range(W)]) for ell in range(N + 1)]


def _errors(kl, g):
    N = g.shape[0] - 1
    err = []
    for ell in range(N + 1):
        for q in range(N + 1):
            e = int(g[ell, 2 * q])
            if e > 0:
                err.append(kl[ell, q] - math.log(e))
            else:
                assert kl[ell, q] == -np.inf, (ell, q)
    return np.abs(np.array(err))


def test_c1_support_and_accuracy_as_configured():
    """4x4, all 17 lines, one walker, seed 1, ln f 1 -> 1e-6, 80% flatness, C = 16N.

    Every reachable bin is visited and nothing else (ergodicity); the error
    of this short, single-walker run is dominated by the ends of the spectrum
    and is bounded loosely here (measured: mean 0.118, max 0.60)."""
    bf = exact.brute_force(4)
    lines = _run_lines(4, [1], 1e-6, 0)
    kl, gk = oracle.assemble(4, lines)
    err = _errors(kl, bf)
    assert err.mean() <= 0.15 and err.max() <= 0.7


def test_converges_to_exact_dos_L4():
    """With long flatness intervals the walk meets mean <= 0.01, max <= 0.05 in ln g."""
    bf = exact.brute_force(4)
    lines = _run_lines(4, [1, 2, 3, 4], 1e-6, 16384 * 16)
    kl, gk = oracle.assemble(4, lines)
    err = _errors(kl, bf)
    assert err.mean() <= 0.01 and err.max() <= 0.05
    # zero-field marginal against the exact g_k
    ex = exact.log_kaufman_gk(4)[::2]
    m = np.isfinite(ex)
    assert np.all(np.isneginf(gk[~m]))
    e2 = np.abs(gk[m] - ex[m])
    assert e2.mean() <= 0.01 and e2.max() <= 0.05


def test_assemble_invariants():
    L, N = 4, 16
    rng = np.random.default_rng(3)
    lines = []
    for ell in range(N // 2 + 1):
        nb = 2 * min(ell, N - ell) + 1
        a = rng.normal(size=(3, nb)) * 5
        a[:, ::3] = -np.inf if nb > 1 else a[:, ::3]
        if nb == 1:
            a[:] = 0.0
        lines.append(a)
    kl, gk = oracle.assemble(L, lines, n_lines=N // 2 + 1)
    for ell in range(N + 1):
        row = kl[ell]
        fin = row[np.isfinite(row)]
        mx = fin.max()
        assert abs(mx + math.log(np.exp(fin - mx).sum()) - oracle.log_binomial(N, ell)) < 1e-12
        assert np.array_equal(row, kl[N - ell])
    for q in range(N + 1):
        col = kl[:, q][np.isfinite(kl[:, q])]
        if col.size:
            mx = col.max()
            assert abs(gk[q] - (mx + math.log(np.exp(col - mx).sum()))) < 1e-12
        else:
            assert gk[q] == -np.inf


def _exact_lines_L4():
    """Exact ln g(k, ell) of the 4x4 torus per line, bin q <-> k = 2q (brute force)."""
    g = exact.brute_force(4)
    out = []
    for ell in range(9):
        nb = 2 * min(ell, 16 - ell) + 1
        row = np.array([math.log(g[ell, 2 * q]) if g[ell, 2 * q] > 0 else -np.inf for q in range(nb)])
        out.append(row)
    return out


def test_assemble_walker_mean_cancels_antisymmetric_errors():
    """Walkers of one line are averaged in ln g after each is put through
    Eq. 4 (reading R12).  Two walkers whose ln g errors are equal and
    opposite, each offset by an arbitrary constant, must therefore assemble
    to the exact degeneracies: averaging g instead of ln g leaves
    log cosh(error) in every bin, and dropping the final renormalisation
    leaves a per-line offset, so either mistake fails against brute force."""
    rng = np.random.default_rng(11)
    ex = _exact_lines_L4()
    lines = []
    for ell, row in enumerate(ex):
        fin = np.isfinite(row)
        d = np.where(fin, rng.normal(0.0, 0.7, row.size), 0.0)
        lines.append(np.stack([row + d + rng.normal(0, 30), row - d + rng.normal(0, 30)]))
    kl, gk = oracle.assemble(4, lines, n_lines=9)
    for ell, row in enumerate(ex):
        got = kl[ell, :row.size]
        assert np.array_equal(np.isfinite(got), np.isfinite(row))
        fin = np.isfinite(row)
        assert np.abs(got[fin] - row[fin]).max() < 1e-12, ell
    ref = exact.brute_force(4).sum(axis=0)[0::2]
    fin = ref > 0
    assert np.abs(gk[fin] - np.log(ref[fin])).max() < 1e-12


def test_assemble_walker_supports_are_averaged_separately():
    """A bin seen by only some walkers takes its mean over those walkers
    (reading R12), each walker normalised by Eq. 4 over its own support: one
    exact walker plus one that never entered the most populated bin of the
    half-filled line and is otherwise exact up to a constant.  The second
    walker's Eq. 4 offset over its support, log(C / (C - g_top)), is then
    known in closed form, and so is the assembled line.  Averaging before
    normalising, or over all walkers with the missing bin as zero, gives
    other values."""
    ex = _exact_lines_L4()
    ell = 8
    row = ex[ell]
    top = int(np.argmax(row))
    part = row.copy()
    part[top] = -np.inf                                  # never entered
    lines = [np.stack([r, r]) for r in ex]
    lines[ell] = np.stack([row, part + 4.0])
    kl, _ = oracle.assemble(4, lines, n_lines=9)
    got = kl[ell, :row.size]
    C = oracle.log_binomial(16, 8)
    fin = np.isfinite(part)
    # walker 2 after Eq. 4 on its own support: exact + log(C / (C - g_top))
    off = C - math.log(math.exp(C) - math.exp(row[top]))
    mean = np.where(fin, row + off / 2.0, row)           # mean over the walkers that saw each bin
    mx = mean.max()
    expect = mean - (mx + math.log(np.exp(mean - mx).sum())) + C
    assert np.array_equal(np.isfinite(got), np.isfinite(expect))
    both = np.isfinite(expect)
    assert np.abs(got[both] - expect[both]).max() < 1e-12
    assert abs(off) > 0.1                                # the case separates the readings


# --- extra resets at unchanged f (reset_checks) -----------------------------

def _h_sum(w):
    return int(w.state().h.sum())


def test_reset_checks_zero_is_the_plain_walk():
    a = oracle.Walker(6, 13, 5, walker=1, lnf_min=1e-3)
    b = oracle.Walker(6, 13, 5, walker=1, lnf_min=1e-3, reset_checks=0)
    a.advance(200000)
    b.advance(200000)
    sa, sb = a.state(), b.state()
    assert sa.attempts == sb.attempts and sa.stages == sb.stages and sa.k == sb.k
    assert np.array_equal(sa.lng.view(np.uint64), sb.lng.view(np.uint64))
    assert np.array_equal(sa.h, sb.h)


def test_reset_every_failed_test_clears_h_keeps_f():
    """flatness 1.0 is never met on a line with several bins, so with
    reset_checks = 1 every test resets: right after a test h is all zero, ln f
    and the stage count are unchanged and ln g is shifted to min 0."""
    L, ell = 6, 14
    C = 16 * L * L
    w = oracle.Walker(L, ell, 3, flatness=1.0, lnf_min=1e-3, reset_checks=1)
    for m in range(1, 6):
        w.advance(C - 1)
        assert _h_sum(w) == C - 1                 # proposals since the last reset
        w.advance(1)
        s = w.state()
        assert s.attempts == m * C and s.stages == 0 and s.lnf == 1.0
        assert int(s.h.sum()) == 0 and w.info().nfail == 0
        vis = s.vis > 0
        assert vis.sum() > 1 and s.lng[vis].min() == 0.0


def test_reset_after_two_failed_tests():
    L, ell = 6, 14
    C = 16 * L * L
    w = oracle.Walker(L, ell, 3, flatness=1.0, lnf_min=1e-3, reset_checks=2)
    w.advance(C)
    assert _h_sum(w) == C and w.info().nfail == 1     # first failure: no reset yet
    w.advance(C)
    assert _h_sum(w) == 0 and w.info().nfail == 0     # second: reset
    w.advance(C)
    assert _h_sum(w) == C and w.info().nfail == 1


def test_reset_is_the_min_shift_of_the_updated_ln_g():
    """At the test that resets, ln g is that after the proposal's update (the
    current bin += ln f) shifted by its minimum over the visited bins."""
    L, ell = 6, 14
    C = 16 * L * L
    w = oracle.Walker(L, ell, 8, flatness=1.0, lnf_min=1e-3, reset_checks=1)
    w.advance(3 * C - 1)
    before = w.state()
    w.advance(1)
    after = w.state()
    lng = before.lng.copy()
    vis = before.vis.copy()
    q = after.k // 2
    lng[q] = lng[q] + before.lnf          # the last proposal's update (vis[q] may be new)
    vis[q] = 1
    vis = vis > 0
    mn = lng[vis].min()
    expect = np.where(vis, lng - mn, lng)
    assert np.array_equal(expect[vis].view(np.uint64), after.lng[vis].view(np.uint64))


def _state_bits(w):
    s = w.state()
    return (s.attempts, s.accepts, s.stages, s.done, s.k, s.nprev, np.float64(s.lnf).view(np.uint64),
            s.lng.view(np.uint64).tobytes(), s.h.tobytes(), s.vis.tobytes(), s.spins.tobytes(),
            s.up.tobytes(), s.dn.tobytes())


@pytest.mark.parametrize("kw", [dict(L=4, ell=5, check_interval=64),
                                dict(L=6, ell=9, check_interval=100, reset_checks=2),
                                dict(L=4, ell=6, check_interval=48, boundary=1),
                                dict(L=4, ell=7, check_interval=80, lattice=1),
                                dict(L=4, ell=4, check_interval=64, boundary=2)])
def test_walk_is_the_same_in_any_chunks(kw):
    """The walker's state captures the whole walk: advancing by the pieces of
    any split of the proposals (across flatness tests, their boundaries
    exactly and one off, stage changes and the end) gives the state of one
    advance, bit for bit; advancing a finished walker changes nothing."""
    C = kw["check_interval"]
    whole = oracle.Walker(seed=5, lnf_min=1e-3, **kw)
    whole.advance()
    total = whole.info().attempts
    assert whole.info().done and whole.info().stages >= 3
    rng = np.random.default_rng(kw["L"] * 100 + kw["ell"])
    for split in range(3):
        w = oracle.Walker(seed=5, lnf_min=1e-3, **kw)
        done_at = 0
        while not w.info().done:
            if split == 0:
                n = int(rng.integers(1, 3 * C))
            elif split == 1:
                n = C - 1 + (done_at % 3)            # C - 1, C, C + 1 in turn
            else:
                n = 1 if done_at % 50 else int(rng.integers(1, 20 * C))
            w.advance(n)
            done_at += 1
        assert _state_bits(w) == _state_bits(whole), split
    before = _state_bits(whole)
    whole.advance(1000)
    assert _state_bits(whole) == before and whole.info().attempts == total
