"""Pins of the oracle on the triangular and honeycomb lattices.

The method only needs the bonds of the lattice: k counts antiparallel
nearest-neighbour pairs whatever the geometry, and the line walk, the
acceptance rule and the assembly are unchanged.  The paper remarks that the
approach carries over to other lattices and interactions; the two
geometries here live on the same L x L grid of sites:
* triangular: the square lattice's bonds plus one diagonal, (r, c)-(r+1, c+1),
  degree 6;
* honeycomb in brick-wall form: every horizontal bond, and the vertical bond
  below (r, c) only when r + c is even, degree 3.
The references are pinned independently of the oracle's C geometry:
* bond counts against closed forms (periodic 3N and 3N/2; open
  2L(L-1) + (L-1)^2 and L(L-1) + L(L-1)/2), degrees, triangles per bond on
  the triangular torus and bipartiteness of the honeycomb;
* the brute-force g(ell, k) over all 2^16 states of the 4 x 4 lattices
  against hand counts: one up spin breaks z bonds (N ways on a torus; on
  the open lattices as many as its site's hand-counted degree);
  two up spins break 2z - 2 bonds when adjacent (N_B pairs) and 2z
  otherwise; every line sums to C(N, ell); ell <-> N - ell symmetry; k
  even on the triangular torus (even degree), k = ell (mod 2) on the
  honeycomb torus (odd degree);
* the oracle's k from scratch equal to a recount over the Python bond list
  for random configurations;
* the walk recounts k from scratch after every accepted move (debug mode),
  and the assembled DOS of complete runs converges to brute force within
  mean 0.01 / max 0.05 in ln g;
* the Eq. 2 thermodynamics on the assembled plane equal the spin
  enumeration of the Eq. 1 Hamiltonian with these bonds.
"""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from oracle import exact, thermo

TRI, HONEY = oracle.TRIANGULAR, oracle.HONEYCOMB


def _closed_form_bonds(L, lattice, boundary):
    N = L * L
    if lattice == TRI:
        return 2 * L * (L - 1) + (L - 1) ** 2 if boundary else 3 * N
    return L * (L - 1) + L * (L - 1) // 2 if boundary else 3 * N // 2


@pytest.mark.parametrize("L", [4, 6, 8])
@pytest.mark.parametrize("lattice", [TRI, HONEY])
@pytest.mark.parametrize("boundary", [0, 1])
def test_bond_counts_and_degrees(L, lattice, boundary):
    bl = exact.bonds(L, boundary, lattice)
    nb = _closed_form_bonds(L, lattice, boundary)
    assert len(bl) == nb == oracle.n_bonds(L, boundary, lattice)
    deg = np.zeros(L * L, dtype=int)
    for i, j in bl:
        assert i != j
        deg[i] += 1
        deg[j] += 1
    z = 6 if lattice == TRI else 3
    if not boundary:
        assert (deg == z).all()
    else:
        assert deg.max() == z and deg.min() >= 1 and deg.sum() == 2 * nb


def test_triangular_torus_triangles():
    """Every bond of the periodic triangular lattice lies on exactly two
    triangles (the faces on either side of it)."""
    L = 6
    bl = exact.bonds(L, 0, TRI)
    adj = [set() for _ in range(L * L)]
    for i, j in bl:
        adj[i].add(j)
        adj[j].add(i)
    for i, j in bl:
        assert len(adj[i] & adj[j]) == 2


@pytest.mark.parametrize("boundary", [0, 1])
def test_honeycomb_bipartite(boundary):
    """The brick wall is bipartite with colour (r + c) mod 2 (L even keeps
    that across the periodic wrap): no odd cycle, as on the honeycomb."""
    L = 6
    for i, j in exact.bonds(L, boundary, HONEY):
        ri, ci = divmod(i, L)
        rj, cj = divmod(j, L)
        assert (ri + ci) % 2 != (rj + cj) % 2


@pytest.fixture(scope="module", params=[(TRI, 0), (TRI, 1), (HONEY, 0), (HONEY, 1)],
                ids=["tri-periodic", "tri-open", "honey-periodic", "honey-open"])
def geo_bf(request):
    lattice, boundary = request.param
    return lattice, boundary, exact.brute_force(4, boundary, lattice)


def test_bruteforce_hand_counts(geo_bf):
    lattice, boundary, g = geo_bf
    L, N = 4, 16
    NB = _closed_form_bonds(L, lattice, boundary)
    assert g.shape == (N + 1, NB + 1)
    assert g.sum() == 1 << N
    for ell in range(N + 1):
        assert g[ell].sum() == math.comb(N, ell)
        assert np.array_equal(g[ell], g[N - ell])
    assert g[0, 0] == 1 and g[0].sum() == 1
    if not boundary:
        z = 6 if lattice == TRI else 3
        assert g[1, z] == N and g[1].sum() == N
        assert g[2, 2 * z - 2] == NB and g[2, 2 * z] == math.comb(N, 2) - NB
        assert g[2].sum() == g[2, 2 * z - 2] + g[2, 2 * z]
        if lattice == TRI:
            assert not g[:, 1::2].any()                      # even degree: k even
        else:
            for ell in range(N + 1):                         # odd degree: k = ell (mod 2)
                assert not g[ell, (ell + 1) % 2::2].any()
    else:
        assert g[:, 1::2].any()
        # One up spin breaks as many bonds as its site has neighbours; the
        # degrees of the open 4 x 4 lattices counted by hand.  Triangular:
        # two corners of degree 2 ((0, 3), (3, 0)), two of degree 3 ((0, 0),
        # (3, 3)), eight edge sites of degree 4, four interior sites of 6.
        # Brick wall: ends of rows have one horizontal bond, and the vertical
        # one goes down from r + c even (not from the last row) and up from
        # r + c odd (not from the first): degrees 1 at (0, 3), (3, 3); 3 at
        # (0, 2), (1, 1), (1, 2), (2, 1), (2, 2), (3, 2); 2 elsewhere.
        want = {2: 2, 3: 2, 4: 8, 6: 4} if lattice == TRI else {1: 2, 2: 8, 3: 6}
        assert {k: int(v) for k, v in enumerate(g[1]) if v} == want


@pytest.mark.parametrize("lattice", [TRI, HONEY])
@pytest.mark.parametrize("boundary", [0, 1])
def test_count_k_matches_bond_list(lattice, boundary):
    rng = np.random.default_rng(11 + lattice + 5 * boundary)
    L = 6
    bl = np.array(exact.bonds(L, boundary, lattice))
    for _ in range(40):
        s = (rng.random(L * L) < rng.random()).astype(np.uint8)
        ref = int((s[bl[:, 0]] != s[bl[:, 1]]).sum())
        assert oracle.count_k(L, s, boundary, lattice) == ref


@pytest.mark.parametrize("lattice", [TRI, HONEY])
@pytest.mark.parametrize("boundary", [0, 1])
@pytest.mark.parametrize("L,ell", [(4, 1), (4, 7), (6, 13), (8, 32)])
def test_walk_recount_and_consistency(lattice, boundary, L, ell):
    N = L * L
    w = oracle.Walker(L, ell, seed=5, walker=2, lnf_min=1e-4, check_interval=64 * N, debug=True,
                      boundary=boundary, lattice=lattice)
    shift = oracle.bin_shift(boundary, lattice)
    z = 6 if lattice == TRI else 3
    for _ in range(10):
        w.advance(4000)                   # raises if the debug recount disagrees
        s = w.state()
        assert s.k == oracle.count_k(L, s.spins, boundary, lattice)
        assert sorted(s.up.tolist()) == np.flatnonzero(s.spins == 1).tolist()
        assert 0 <= s.k <= min(z * min(ell, N - ell), oracle.n_bonds(L, boundary, lattice))
        assert s.nb == oracle.n_bins(L, ell, boundary, lattice)
        assert s.nb == (min(z * min(ell, N - ell), oracle.n_bonds(L, boundary, lattice)) >> shift) + 1
        if s.done:
            break


def _run_lines(L, seeds, lnf_min, C, boundary, lattice):
    N = L * L
    jobs = [(ell, s) for ell in range(N // 2 + 1) for s in seeds]
    with ThreadPoolExecutor(8) as pool:
        res = list(pool.map(lambda j: oracle.line_run(L, j[0], j[1], lnf_min=lnf_min, check_interval=C,
                                                      boundary=boundary, lattice=lattice), jobs))
    W = len(seeds)
    return [np.stack([res[ell * W + i][0] for i in range(W)]) for ell in range(N // 2 + 1)]


def test_converges_to_exact_dos_L4(geo_bf):
    """Long flatness intervals: mean <= 0.01, max <= 0.05 in ln g, every
    reachable (k, ell) visited and nothing else."""
    lattice, boundary, g = geo_bf
    L, N = 4, 16
    lines = _run_lines(L, [1, 2, 3, 4], 1e-6, 1 << 20, boundary, lattice)
    kl, gk = oracle.assemble(L, lines, boundary=boundary, lattice=lattice)
    ref = thermo.lng_from_counts(g, boundary, lattice)
    assert kl.shape == ref.shape
    sup = np.isfinite(ref)
    assert np.array_equal(np.isfinite(kl), sup)
    err = np.abs(kl[sup] - ref[sup])
    assert err.mean() <= 0.01 and err.max() <= 0.05
    tot = thermo.lng_from_counts(g.sum(axis=0, keepdims=True), boundary, lattice)[0]
    assert np.array_equal(np.isfinite(gk), np.isfinite(tot))
    assert np.abs(gk[np.isfinite(tot)] - tot[np.isfinite(tot)]).max() <= 0.05


@pytest.mark.parametrize("beta,H,J", [(0.3, 0.2, 1.0), (0.7, -0.3, -1.0)])
def test_thermodynamics_equal_spin_enumeration(geo_bf, beta, H, J):
    lattice, boundary, g = geo_bf
    lng = thermo.lng_from_counts(g, boundary, lattice)
    got = thermo.thermo(4, lng, beta, H, J, boundary, lattice)
    ref = thermo.spin_enumeration(4, beta, H, J, boundary, lattice)
    for f in thermo.FIELDS:
        assert got[f] == pytest.approx(ref[f], rel=1e-11, abs=1e-12), f


@pytest.mark.parametrize("beta,H", [(0.3, 0.4), (1.1, -0.25)])
def test_independent_spins_J0_on_every_lattice(geo_bf, beta, H):
    """J = 0 leaves independent spins in a field whatever the bonds:
    ln Z = N ln 2 cosh(beta H), m = tanh(beta H), chi = beta (1 - m^2)."""
    lattice, boundary, g = geo_bf
    N = 16
    got = thermo.thermo(4, thermo.lng_from_counts(g, boundary, lattice), beta, H, 0.0, boundary, lattice)
    m = math.tanh(beta * H)
    assert got["lnZ"] == pytest.approx(N * math.log(2.0 * math.cosh(beta * H)), rel=1e-12)
    assert got["m"] == pytest.approx(m, rel=1e-10, abs=1e-13)
    assert got["chi"] == pytest.approx(beta * (1.0 - m * m), rel=1e-9)


def test_ground_state_energy_of_the_ferromagnet(geo_bf):
    """At low temperature and J = 1, H = 0 the energy per spin tends to
    -N_B / N (every bond satisfied): -3 on the triangular torus, -1.5 on the
    honeycomb torus, the bond count over N on the open lattices."""
    lattice, boundary, g = geo_bf
    NB = _closed_form_bonds(4, lattice, boundary)
    got = thermo.thermo(4, thermo.lng_from_counts(g, boundary, lattice), 12.0, 0.0, 1.0, boundary, lattice)
    assert got["e"] == pytest.approx(-NB / 16.0, rel=1e-6)
