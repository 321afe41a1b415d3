"""Pins of the oracle on a model without up-down symmetry: the periodic
lattice with its last row of L spins held up (boundary 2).  Lines ell count
up spins among the N - L free sites and run 0..N - L; no line follows from
another by flipping every spin, so the assembly takes all of them (the
paper's remark that asymmetric models need every line, twice the work of
the symmetric case).

The exact reference is brute force over the 2^12 free configurations of
the 4 x 4 lattice, itself pinned by hand counts:
* every line sums to C(N - L, ell), the whole table to 2^(N - L);
* ell = 0: the held row against two down rows, k = 2L; ell = N - L: k = 0;
* one free up spin: next to the held row (rows 0 and L - 2, 2L sites) it
  breaks 3 bonds and heals 1, k = 2L + 2; elsewhere ((L - 3) L sites) it
  breaks 4, k = 2L + 4;
* the table differs from its mirror g(k, N - L - ell).
The walk itself: every accepted move is recounted from scratch (debug mode),
the held row never moves, and with long flatness intervals the assembled DOS
converges to brute force within the bounds used elsewhere.
"""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from oracle import exact

HELD = oracle.HELD


@pytest.fixture(scope="module")
def bfh():
    return exact.brute_force(4, boundary=HELD)


def test_bruteforce_held_counts(bfh):
    L, N = 4, 16
    Nf = N - L
    assert bfh.shape == (N + 1, 2 * N + 1)
    assert bfh.sum() == 1 << Nf
    for ell in range(Nf + 1):
        assert bfh[ell].sum() == math.comb(Nf, ell)
    assert not bfh[Nf + 1:].any()
    assert bfh[0, 2 * L] == 1 and bfh[0].sum() == 1
    assert bfh[Nf, 0] == 1 and bfh[Nf].sum() == 1
    assert bfh[1, 2 * L + 2] == 2 * L and bfh[1, 2 * L + 4] == (L - 3) * L and bfh[1].sum() == Nf
    assert not bfh[:, 1::2].any()                       # k even on the periodic lattice
    mirror = bfh[Nf::-1]
    assert not np.array_equal(bfh[:Nf + 1], mirror)     # no up-down symmetry


def test_held_bins_cover_the_reachable_k(bfh):
    L, N = 4, 16
    for ell in range(N - L + 1):
        nb = oracle.n_bins(L, ell, HELD)
        ks = np.flatnonzero(bfh[ell])
        assert ks.max() >> 1 < nb
        assert nb == min(2 * min(ell + L, N - L - ell), N) + 1


@pytest.mark.parametrize("L,ell", [(4, 1), (4, 6), (4, 11), (6, 9), (6, 20), (8, 7), (8, 30), (10, 47)])
def test_held_walk_recount_and_consistency(L, ell):
    N = L * L
    Nf = N - L
    w = oracle.Walker(L, ell, seed=78, walker=2, lnf_min=1e-4, check_interval=64 * N, debug=True, boundary=HELD)
    for _ in range(20):
        w.advance(5000)                  # raises if the debug recount disagrees
        s = w.state()
        assert s.k == oracle.count_k(L, s.spins, boundary=HELD)
        assert (s.spins[Nf:] == 1).all()                       # the held row never moves
        assert sorted(s.up.tolist()) == np.flatnonzero(s.spins[:Nf] == 1).tolist()
        assert sorted(s.dn.tolist()) == np.flatnonzero(s.spins[:Nf] == 0).tolist()
        assert s.up.size == ell and s.dn.size == Nf - ell
        assert s.nb == oracle.n_bins(L, ell, HELD)
        if s.done:
            break


def test_held_edge_lines_and_bad_ell():
    L, N = 4, 16
    lng, info = oracle.line_run(L, 0, seed=1, boundary=HELD)
    assert info.done == 1 and np.isfinite(lng).sum() == 1 and lng[L] == 0.0     # k = 2L, bin L
    lng, info = oracle.line_run(L, N - L, seed=1, boundary=HELD)
    assert info.done == 1 and lng[0] == 0.0
    with pytest.raises(ValueError):
        oracle.line_run(L, N - L + 1, seed=1, boundary=HELD)


def _run_lines_held(L, seeds, lnf_min, C):
    Nf = L * L - L
    jobs = [(ell, s) for ell in range(Nf + 1) for s in seeds]
    with ThreadPoolExecutor(8) as pool:
        res = list(pool.map(lambda j: oracle.line_run(L, j[0], j[1], lnf_min=lnf_min, check_interval=C,
                                                      boundary=HELD), jobs))
    W = len(seeds)
    return [np.stack([res[ell * W + i][0] for i in range(W)]) for ell in range(Nf + 1)]


def test_held_converges_to_exact_dos_L4(bfh):
    """Long flatness intervals: mean <= 0.01, max <= 0.05 in ln g, every
    reachable (k, ell) visited and nothing else; the assembly of all 13
    lines (no mirroring) and its zero-field marginal."""
    L, N = 4, 16
    lines = _run_lines_held(L, [1, 2, 3, 4], 1e-6, 16384 * N)
    kl, gk = oracle.assemble(L, lines, boundary=HELD)
    assert kl.shape == (N + 1, N + 1)
    err = []
    for ell in range(N + 1):
        for q in range(N + 1):
            c = bfh[ell, 2 * q]
            if c > 0:
                err.append(abs(kl[ell, q] - math.log(c)))
            else:
                assert kl[ell, q] == -np.inf, (ell, q)
    err = np.array(err)
    assert err.mean() <= 0.01 and err.max() <= 0.05
    tot = bfh.sum(axis=0)[0::2]
    assert np.all(np.isneginf(gk[tot == 0]))
    assert np.abs(gk[tot > 0] - np.log(tot[tot > 0])).max() <= 0.05


def test_held_assembly_requires_every_line():
    L = 4
    lines = [np.zeros((1, oracle.n_bins(L, e, HELD))) for e in range(L * L // 2 + 1)]
    with pytest.raises(ValueError):
        oracle.assemble(L, lines, boundary=HELD)
