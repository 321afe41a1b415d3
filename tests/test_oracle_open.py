"""Pins of the oracle with open boundaries (free edges: no bond across them).

The exact reference is brute force over all 2^16 states of the open 4 x 4
lattice, itself pinned by hand counts:
* N_B = 2L(L-1) bonds; every line sums to C(N, ell); ell <-> N - ell symmetry.
* One up spin: in a corner it breaks 2 bonds, on an edge 3, inside 4, so the
  ell = 1 line is g(2) = 4, g(3) = 4(L-2), g(4) = (L-2)^2.
* Half the spins up with the fewest broken bonds: a straight cut through
  the lattice, k = L, four ways (two orientations, two colourings).
The walk itself: every accepted move is recounted from scratch (debug mode),
k can be odd, and with long flatness intervals the assembled DOS converges
to brute force within the bounds used for the periodic lattice.  The
thermodynamics of Eq. 2 with N_B = 2L(L-1) equal the open-lattice spin
enumeration.
"""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from oracle import exact, thermo


@pytest.fixture(scope="module")
def bfo():
    return exact.brute_force(4, boundary=1)


def test_bruteforce_open_counts(bfo):
    L, N = 4, 16
    assert bfo.shape == (N + 1, 2 * L * (L - 1) + 1)
    assert bfo.sum() == 1 << N
    for ell in range(N + 1):
        assert bfo[ell].sum() == math.comb(N, ell)
        assert np.array_equal(bfo[ell], bfo[N - ell])
    assert bfo[1, 2] == 4 and bfo[1, 3] == 4 * (L - 2) and bfo[1, 4] == (L - 2) ** 2
    assert bfo[1].sum() == bfo[1, 2] + bfo[1, 3] + bfo[1, 4]
    assert not bfo[N // 2, :L].any() and bfo[N // 2, L] == 4
    assert bfo[:, 1::2].any()                   # odd k occur on the open lattice


def test_count_k_open_matches_enumeration():
    rng = np.random.default_rng(4)
    L = 6
    for _ in range(50):
        s = (rng.random(L * L) < 0.5).astype(np.uint8)
        ref = 0
        for r in range(L):
            for c in range(L):
                if c + 1 < L:
                    ref += s[r * L + c] != s[r * L + c + 1]
                if r + 1 < L:
                    ref += s[r * L + c] != s[(r + 1) * L + c]
        assert oracle.count_k(L, s, boundary=1) == ref


@pytest.mark.parametrize("L,ell", [(4, 1), (4, 5), (4, 8), (6, 9), (6, 18), (8, 7), (8, 32), (10, 47)])
def test_open_walk_recount_and_consistency(L, ell):
    N = L * L
    w = oracle.Walker(L, ell, seed=77, walker=1, lnf_min=1e-4, check_interval=64 * N, debug=True, boundary=1)
    odd = False
    for _ in range(20):
        w.advance(5000)                  # raises if the debug recount disagrees
        s = w.state()
        assert s.k == oracle.count_k(L, s.spins, boundary=1)
        assert sorted(s.up.tolist()) == np.flatnonzero(s.spins == 1).tolist()
        assert 0 <= s.k <= min(4 * min(ell, N - ell), 2 * L * (L - 1))
        assert s.nb == oracle.n_bins(L, ell, 1)
        odd |= bool(np.any(s.vis[1::2]))
        if s.done:
            break
    assert odd                           # bins of odd k are visited


def test_open_edge_lines():
    L, N = 4, 16
    lng, info = oracle.line_run(L, 1, seed=1, boundary=1)
    assert lng.size == 5 and np.isinf(lng[0]) and np.isinf(lng[1]) and np.isfinite(lng[2:]).all()
    lng, info = oracle.line_run(L, 0, seed=1, boundary=1)
    assert lng.tolist() == [0.0] and info.done == 1


def _run_lines_open(L, seeds, lnf_min, C):
    N = L * L
    jobs = [(ell, s) for ell in range(N + 1) for s in seeds]
    with ThreadPoolExecutor(8) as pool:
        res = list(pool.map(lambda j: oracle.line_run(L, j[0], j[1], lnf_min=lnf_min, check_interval=C,
                                                      boundary=1), jobs))
    W = len(seeds)
    return [np.stack([res[ell * W + i][0] for i in range(W)]) for ell in range(N + 1)]


def test_open_converges_to_exact_dos_L4(bfo):
    """Long flatness intervals: mean <= 0.01, max <= 0.05 in ln g, every
    reachable (k, ell) visited and nothing else."""
    lines = _run_lines_open(4, [1, 2, 3, 4], 1e-6, 16384 * 16)
    kl, gk = oracle.assemble(4, lines, boundary=1)
    assert kl.shape == (17, 25)
    err = []
    for ell in range(17):
        for k in range(25):
            if bfo[ell, k] > 0:
                err.append(abs(kl[ell, k] - math.log(bfo[ell, k])))
            else:
                assert kl[ell, k] == -np.inf, (ell, k)
    err = np.array(err)
    assert err.mean() <= 0.01 and err.max() <= 0.05
    tot = bfo.sum(axis=0)
    assert np.all(np.isneginf(gk[tot == 0]))
    assert np.abs(gk[tot > 0] - np.log(tot[tot > 0])).max() <= 0.05


@pytest.mark.parametrize("beta,H,J", [(0.3, 0.2, 1.0), (0.8, -0.4, 1.0), (0.5, 0.1, -1.0)])
def test_open_thermodynamics_equal_spin_enumeration(bfo, beta, H, J):
    lng = thermo.lng_from_counts(bfo, boundary=1)
    got = thermo.thermo(4, lng, beta, H, J, boundary=1)
    ref = thermo.spin_enumeration(4, beta, H, J, boundary=1)
    for f in thermo.FIELDS:
        assert got[f] == pytest.approx(ref[f], rel=1e-11, abs=1e-12), f


def test_open_line_edges_as_the_paper_states(bfo):
    """Discussion of Figs. 1-2 with free edges (N_B = 2L(L-1)): the half-filled
    line's lowest k is one straight interface of L bonds (the four cuts
    through the middle of the 4x4), so its ground state lies at
    k/N_B = 1/(2(L-1)); its top is the two Neel states at k = N_B.  A line
    reaches k = 4 ell only while its up spins fit pairwise apart on interior
    sites (four bonds each: a 2x2 block at L = 4, room for two), and stays
    below 4 ell beyond, approaching the periodic levels only as L grows."""
    L, N = 4, 16
    NB = 2 * L * (L - 1)
    half = bfo[N // 2]
    ks = np.nonzero(half)[0]
    assert ks.min() == L and half[L] == 4 and ks.min() / NB == 1 / (2 * (L - 1))
    assert ks.max() == NB and half[NB] == 2
    for ell in range(1, N // 2 + 1):
        top = np.nonzero(bfo[ell])[0].max()
        assert (top == 4 * ell) == (ell <= 2), ell
        assert top <= 4 * ell
