"""Late-stage parity with the oracle in the launch configurations the
benchmark and the completion runs use.

The walks are taken past flatness tests, stage transitions and walker
completion in:
  - the 64x64 throughput workload (every walker L = 64, which selects the
    kernel specialised for that shape) over sixteen launches of 65536
    proposals, sampling the lines ell = 1, 2, 3 (which finish or transition
    inside the window) and the widest lines;
  - the 256x256 workload in its benchmark launches (16384 proposals each)
    past the first two flatness tests (C = 16N = 2^20);
  - 16x16 and 32x32 lines run to ln f < 1e-5 with the switch of the last
    walkers to one wavefront each in the middle of the run, so that the
    row form of that kernel works through the late stages.
The complete walker state must equal the oracle's bit for bit (the line-walk
paragraph and Eq. 3-4 of the paper define every step).  The device's
acceptance exponential is compared with the oracle's on a grid.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from _progress import say

import oracle
from paper_1302_2320_amd import wl, workloads
from paper_1302_2320_amd.workloads import LineSpec

pytestmark = pytest.mark.gpu


def _say(msg):
    say(msg)


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
    tag = f"walker {idx} (L={p.L} ell={p.ell} seed={p.seed} w={p.walker})"
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


@pytest.mark.parametrize("placement", [0, 6, 8])
def test_l64_sixteen_launches_bitwise(placement):
    """16 launches of 65536 proposals of the 64x64 workload: ell = 1 finishes
    (14 stages at one test each, 14 * 16N < 2^20 proposals), ell = 2, 3
    transition; the widest lines (ell = 2047, 2048) are sampled as well.
    Placement 0 is the library's choice for the workload."""
    lines = workloads.l64()
    S, n = 1 << 16, 16
    _say(f"l64: {len(lines)} walkers, placement {placement}, {n} launches of {S}")
    b = wl.Batch(lines, placement=placement)
    for _ in range(n):
        b.advance(S)
    rng = np.random.default_rng(19)
    must = list(range(8, 32)) + list(range(8 * 2047, 8 * 2049))
    idx = sorted(set(must + [int(x) for x in rng.integers(0, len(lines), 16)]))
    refs = _oracle_states([lines[i] for i in idx], n * S)
    for i, r in zip(idx, refs):
        _compare(b, i, r, lines[i])
    by_ell = {}
    for i, r in zip(idx, refs):
        by_ell.setdefault(lines[i].ell, []).append(r)
    assert all(r.done and r.stages == 14 for r in by_ell[1])
    assert all(r.stages > 0 for r in by_ell[2] + by_ell[3])
    b.close()


def test_c5_past_flatness_tests_bitwise():
    """The 256x256 workload (21.8 GB of walker state) in the benchmark's
    launches of 16384 proposals, 129 of them: every walker passes the tests at
    2^20 and 2^21 proposals; ell = 1 and ell = 2 reduce ln f there."""
    lines = workloads.c5()
    S, n = 1 << 14, 129
    _say(f"c5: {len(lines)} walkers, {n} launches of {S}")
    b = wl.Batch(lines)
    for _ in range(n):
        b.advance(S)
    rng = np.random.default_rng(23)
    must = [0, 1, 2, 3, 4, 16383, 16384, 32767, 32768]
    idx = sorted(set(must + [int(x) for x in rng.integers(0, len(lines), 12)]))
    refs = _oracle_states([lines[i] for i in idx], n * S)
    for i, r in zip(idx, refs):
        _compare(b, i, r, lines[i])
    stages = {lines[i].ell: r.stages for i, r in zip(idx, refs)}
    assert stages[1] == 2 and stages[2] >= 1
    b.close()


def test_tail_switch_late_stages_bitwise():
    """16x16 and 32x32 lines to ln f < 1e-5 (9 stages): lane per walker until
    three walkers are left (after the 16x16 line ell = 37 ends, midway in the
    wider lines' runs), then one wavefront each (row form, N > 64) to the end."""
    lines = [LineSpec(L=16, ell=e, seed=11, lnf_min=1e-5) for e in (1, 2, 37, 90, 128)] + \
            [LineSpec(L=32, ell=e, seed=11, lnf_min=1e-5) for e in (3, 50)]
    _say(f"tail switch: {len(lines)} walkers to ln f < 1e-5, tail_walkers 3")
    b = wl.Batch(lines, tail_walkers=3)
    counts = []
    while True:
        active = b.run(1 << 18, 1)
        counts.append(active)
        if active == 0:
            break
    assert 3 in counts or any(c < 3 for c in counts[:-1])
    refs = _oracle_states(lines, (1 << 64) - 1)
    for i, (p, r) in enumerate(zip(lines, refs)):
        assert r.done and r.stages == 9
        _compare(b, i, r, p)
    b.close()


def test_exp_fixed_device_bitwise():
    """exp_fixed as the walk kernels evaluate it equals the oracle's on a
    dense grid, random arguments and the edges of its range (both follow one
    definition: Cody-Waite reduction, degree-13 Taylor polynomial, 2^n)."""
    rng = np.random.default_rng(5)
    ln2 = np.log(2.0)
    x = np.concatenate([
        np.linspace(-745.0, 0.0, 200001),
        -rng.uniform(0.0, 700.0, 100000),
        -rng.uniform(0.0, 1e-3, 20000),
        -np.exp(rng.uniform(-700.0, 0.0, 20000)),
        np.array([-0.0, 0.0, -700.0, np.nextafter(-700.0, -np.inf), np.nextafter(-700.0, 0.0), -708.4,
                  -745.1, -5e-324, -1e-300, -1e-16, -0.5 * ln2, -ln2, -1.5 * ln2]),
        np.concatenate([[-(j + 0.5) * ln2, np.nextafter(-(j + 0.5) * ln2, 0.0),
                         np.nextafter(-(j + 0.5) * ln2, -np.inf)] for j in range(0, 1000, 7)]),
    ])
    _say(f"exp_fixed on the device: {x.size} arguments")
    got = wl.exp_fixed_device(x).cpu().numpy()
    ref = np.array([oracle.exp_fixed(float(v)) for v in x])
    bad = np.nonzero(_bits(got) != _bits(ref))[0]
    assert bad.size == 0, [(float(x[i]), float(got[i]), float(ref[i])) for i in bad[:5]]
