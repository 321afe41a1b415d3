"""Exact references cross-checked against each other and against counting.

Brute force (all 2^16 states at L = 4), the transfer matrix (L <= 8) and the
Kaufman/Pfaffian zero-field g_k are three independent computations of the
degeneracies of Eq. 2; the closed forms follow by hand-counting.  Agreement
between them pins every exact table the WL oracle is later compared with.
"""
import math

import numpy as np
import pytest

from oracle import exact


@pytest.fixture(scope="module")
def bf4():
    return exact.brute_force(4)


@pytest.fixture(scope="module")
def tm():
    return {L: exact.transfer_matrix(L) for L in (4, 6, 8)}


def test_bruteforce_equals_transfer_matrix_L4(bf4, tm):
    assert np.array_equal(bf4, tm[4].astype(np.int64))


def test_bruteforce_worked_values_L4(bf4):
    # Zero-field and the half-filled line of the 4x4 torus, counted by hand
    # from the structure of the spectrum: g_0 = 2 (both ground states),
    # g_32 = 2 (Neel), the ell = 8 line holds the 2L = 8 stripe states at
    # k = 2L = 8 (the line's ground state) and the two Neel states at k = N_B.
    gk = bf4.sum(axis=0)
    assert gk[0] == 2 and gk[32] == 2 and gk[4] == 32      # one flipped spin: N ways, x2 for the mirror
    assert bf4[8, 8] == 8 and bf4[8, 32] == 2
    assert gk.sum() == 2 ** 16


@pytest.mark.parametrize("L", [4, 6, 8])
def test_transfer_matrix_invariants(tm, L):
    g = tm[L]
    N = L * L
    for ell in range(N + 1):
        row = [int(x) for x in g[ell]]
        # micromagnetic marginal g_ell = C(N, ell)  (Eq. 2 with J = 0)
        assert sum(row) == math.comb(N, ell)
        # up-down symmetry
        assert row == [int(x) for x in g[N - ell]]
        # k is even; support k <= 4 min(ell, N - ell)
        m = min(ell, N - ell)
        for k, v in enumerate(row):
            if v:
                assert k % 2 == 0 and k <= 4 * m
        # k = 0 only for the two uniform states
        assert (row[0] != 0) == (ell in (0, N))
    # ground state of the half-filled line: k = 2L with 2L stripe states; Neel: k = N_B, g = 2
    assert int(g[N // 2, 2 * L]) == 2 * L and int(g[N // 2, 2 * N]) == 2
    assert int(g[N // 2, :2 * L].sum()) == 0
    # top of the spectrum for ell <= N/2 is k = 4 ell (scattered up spins) while those fit
    for ell in range(1, N // 8 + 1):
        assert int(g[ell, 4 * ell]) > 0


@pytest.mark.parametrize("L", [4, 6, 8])
def test_kaufman_equals_sum_over_lines(tm, L):
    g = tm[L]
    N = L * L
    summed = [sum(int(g[ell, k]) for ell in range(N + 1)) for k in range(2 * N + 1)]
    assert list(exact.kaufman_gk(L)) == summed


@pytest.mark.parametrize("L", [4, 6, 8])
def test_closed_forms(tm, L):
    for (k, ell), v in exact.closed_forms(L).items():
        assert int(tm[L][ell, k]) == v, (k, ell)


@pytest.mark.parametrize("L", [10, 16])
def test_kaufman_invariants_larger(L):
    g = exact.kaufman_gk(L)
    N = L * L
    assert sum(g) == 2 ** N
    assert g[0] == 2 and g[2 * N] == 2           # ground states, Neel states
    assert g[4] == 2 * N                         # one flipped spin (or its mirror)
    assert g[6] == 2 * 2 * N                     # an adjacent flipped pair
    assert all(v == 0 for v in g[1::2])          # k even
    assert all(g[k] == g[2 * N - k] for k in range(2 * N + 1))   # bipartite: k <-> N_B - k
    # lowest-k counts agree with the closed forms of the ell <= 3 lines (and mirrors):
    cf = exact.closed_forms(L)
    assert g[8] == 2 * (cf[(8, 2)] + cf[(8, 3)] + _four_in_square(N))
    assert g[2] == 0


def _four_in_square(N):
    # four up spins forming a 2x2 block break 8 bonds; N positions
    return N


@pytest.mark.parametrize("L", [4, 6, 8])
def test_line_tops_end_the_curves_where_the_paper_places_them(tm, L):
    """Discussion of Fig. 1: a line's highest k has every up spin among down
    neighbours only, k = 4 ell, and for ell <= N/2 such placements exist (one
    sublattice holds N/2 sites); on the torus (N_B = 2N) the lines
    ell = N/8, N/4, 3N/8 therefore end at k/N_B = 1/4, 1/2, 3/4."""
    g = tm[L]
    N = L * L
    NB = 2 * N
    tops = {}
    for ell in range(1, N // 2 + 1):
        tops[ell] = max(k for k in range(NB + 1) if int(g[ell, k]))
        assert tops[ell] == 4 * ell
    if N % 8 == 0:
        assert [tops[e] / NB for e in (N // 8, N // 4, 3 * N // 8)] == [0.25, 0.5, 0.75]
