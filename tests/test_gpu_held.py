"""The model without up-down symmetry (the last row held up, boundary 2) on
the device path.

- Walkers with a held row, side by side with ordinary ones, walk the
  oracle's trajectories bit for bit on every placement (the held sites are
  in the lattice but in neither list, so every kernel reads them as up
  neighbours and never flips them), on the square, triangular and honeycomb
  lattices and on two-word rows.
- Lines run to the end through the switch to one wavefront per walker (board
  and row forms) equal the oracle's complete runs.
- The 4x4 DOS from all thirteen lines (no mirroring), walked and assembled on
  the device, equals the oracle's assembly of the oracle's lines and lies
  within mean 0.01 / max 0.05 of brute force over the 2^12 free
  configurations.
"""
import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from _progress import say

import oracle
from oracle import exact
from paper_1302_2320_amd import wl
from paper_1302_2320_amd.workloads import LineSpec

pytestmark = pytest.mark.gpu

HELD = 2


def _bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


def _oracle_state(p, attempts):
    w = oracle.Walker(p.L, p.ell, p.seed, p.walker, p.lnf0, p.lnf_min, p.flatness, p.check_interval,
                      reset_checks=p.reset_checks, boundary=p.boundary, lattice=p.lattice)
    w.advance(attempts)
    return w.state()


def _oracle_states(lines, attempts):
    with ThreadPoolExecutor(8) as pool:
        return list(pool.map(lambda p: _oracle_state(p, attempts), lines))


def _compare(batch, idx, ref, p):
    g = batch.read_walker(idx)
    tag = f"walker {idx} (L={p.L} ell={p.ell} boundary={p.boundary} lattice={p.lattice})"
    assert g.stats["attempts"] == ref.attempts, tag
    assert g.stats["accepts"] == ref.accepts, tag
    assert g.stats["stages"] == ref.stages, tag
    assert bool(g.stats["done"]) == ref.done, tag
    assert g.stats["k"] == ref.k, tag
    assert g.stats["final_lnf"] == ref.lnf, tag
    assert g.nprev == ref.nprev, tag
    assert np.array_equal(_bits(g.lng), _bits(np.where(ref.vis > 0, ref.lng, -np.inf))), tag
    assert np.array_equal(g.h, ref.h), tag
    assert np.array_equal(g.spins, ref.spins), tag
    assert np.array_equal(g.up.astype(np.int32), ref.up), tag
    assert np.array_equal(g.dn.astype(np.int32), ref.dn), tag
    if p.boundary == HELD:
        assert (g.spins[p.L * p.L - p.L:] == 1).all(), tag


def _held_lines(lattices=(0,), sides=(4, 6, 8, 12, 16, 32, 64)):
    out = []
    rng = np.random.default_rng(1302)
    for lattice in lattices:
        for L in sides:
            Nf = L * L - L
            ells = sorted(set([0, 1, 2, Nf // 2, Nf - 1, Nf] + [int(x) for x in rng.integers(0, Nf + 1, 3)]))
            for e in ells:
                out.append(LineSpec(L=L, ell=e, seed=int(rng.integers(1, 2 ** 40)), walker=int(rng.integers(0, 9)),
                                    lnf_min=float(rng.choice([1e-3, 1e-6])),
                                    check_interval=int(rng.choice([0, 100, 999])), boundary=HELD, lattice=lattice))
            # an ordinary walker of the same side next to them
            out.append(LineSpec(L=L, ell=L, seed=5, walker=1, lnf_min=1e-4, check_interval=300, lattice=lattice))
    return out


@pytest.mark.parametrize("wpw,placement", [(0, 0), (64, 1), (64, 2), (16, 3), (0, 4), (0, 5), (0, 6), (0, 7),
                                           (0, 8)])
def test_held_batch_chunked_bitwise(wpw, placement):
    lines = _held_lines()
    chunks = [777, 4096, 20000]
    say(f"held: {len(lines)} walkers, placement {placement}, chunks {chunks}")
    b = wl.Batch(lines, walkers_per_wave=wpw, placement=placement)
    for c in chunks:
        b.advance(c)
    refs = _oracle_states(lines, sum(chunks))
    for i, (p, r) in enumerate(zip(lines, refs)):
        _compare(b, i, r, p)
    b.close()


@pytest.mark.parametrize("wide", [0, 1])
def test_held_other_lattices_and_wide_rows_bitwise(wide):
    lines = _held_lines(lattices=(1, 2), sides=(4, 8, 16)) + _held_lines(sides=(66, 130))
    chunks = [1000, 9000]
    say(f"held, other lattices and wide rows: {len(lines)} walkers, wide_placement {wide}")
    b = wl.Batch(lines, wide_placement=wide)
    for c in chunks:
        b.advance(c)
    refs = _oracle_states(lines, sum(chunks))
    for i, (p, r) in enumerate(zip(lines, refs)):
        _compare(b, i, r, p)
    b.close()


def test_held_lines_to_completion_bitwise():
    """Lane kernels until three walkers are left, then one wavefront each:
    the board form (L = 4, 8: N <= 64) and the row form (L = 10, 12)."""
    lines = [LineSpec(L=L, ell=e, seed=3, walker=w, lnf_min=1e-5, boundary=HELD)
             for L, e in ((4, 5), (8, 17), (8, 40), (10, 33), (12, 70)) for w in (0, 1)]
    say(f"held to completion: {len(lines)} walkers, tail_walkers 3")
    b = wl.Batch(lines, tail_walkers=3)
    while b.run(1 << 18, 1) > 0:
        pass
    refs = _oracle_states(lines, (1 << 64) - 1)
    for i, (p, r) in enumerate(zip(lines, refs)):
        assert r.done
        _compare(b, i, r, p)
    b.close()


def test_held_dos_L4_device_assembly_against_oracle_and_brute_force():
    L, N = 4, 16
    Nf = N - L
    seeds = [1, 2, 3, 4]
    C = 16384 * N
    lines = [LineSpec(L=L, ell=e, seed=s, lnf_min=1e-6, check_interval=C, boundary=HELD)
             for e in range(Nf + 1) for s in seeds]
    say(f"held 4x4 DOS: {len(lines)} walkers, C = 16384 N, to 1e-6")
    b = wl.Batch(lines)
    b.run_to_end()
    packed, _ = b.lng()
    kl, gk = wl.assemble(L, packed, Nf + 1, len(seeds), boundary=HELD)
    kl, gk = kl.cpu().numpy(), gk.cpu().numpy()
    per = b.lng_list()
    b.close()
    # the oracle's lines, assembled by the oracle
    with ThreadPoolExecutor(8) as pool:
        res = list(pool.map(lambda p: oracle.line_run(L, p.ell, p.seed, lnf_min=p.lnf_min,
                                                      check_interval=p.check_interval, boundary=HELD)[0], lines))
    W = len(seeds)
    for i in range(len(lines)):
        assert np.array_equal(_bits(per[i]), _bits(res[i]))
    ref_kl, ref_gk = oracle.assemble(L, [np.stack(res[e * W:(e + 1) * W]) for e in range(Nf + 1)], boundary=HELD)
    assert np.array_equal(np.isinf(kl), np.isinf(ref_kl))
    fin = np.isfinite(ref_kl)
    assert np.max(np.abs(kl[fin] - ref_kl[fin])) < 1e-11
    assert np.max(np.abs(gk[np.isfinite(ref_gk)] - ref_gk[np.isfinite(ref_gk)])) < 1e-11
    # against brute force
    bf = exact.brute_force(L, boundary=HELD)
    err = []
    for ell in range(N + 1):
        for q in range(N + 1):
            c = bf[ell, 2 * q]
            if c > 0:
                err.append(abs(kl[ell, q] - math.log(c)))
            else:
                assert kl[ell, q] == -np.inf, (ell, q)
    err = np.array(err)
    say(f"  |d ln g| mean {err.mean():.4f} max {err.max():.4f}")
    assert err.mean() <= 0.01 and err.max() <= 0.05
    # no up-down symmetry: the table's support differs from its mirror's
    assert not np.array_equal(np.isfinite(kl[:Nf + 1]), np.isfinite(kl[Nf::-1]))
