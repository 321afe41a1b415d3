"""Open boundaries on the GPU (the second lattice the paper runs every
experiment on): bit-exact walker trajectories against the oracle on every
placement, mixed with periodic walkers in one batch, on lattices of one to
three words per row; assembly of open lines (N_B + 1 columns, every k);
thermodynamics of the open plane; the whole 4 x 4 open DOS within the
exact-DOS bounds of brute force."""
import math
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

from _progress import say

import oracle
from oracle import exact, thermo
from paper_1302_2320_amd import wl
from paper_1302_2320_amd.workloads import LineSpec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    say(msg)


def _bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


def _oracle_state(p, attempts):
    w = oracle.Walker(p.L, p.ell, p.seed, p.walker, p.lnf0, p.lnf_min, p.flatness, p.check_interval,
                      reset_checks=p.reset_checks, boundary=p.boundary)
    w.advance(attempts)
    return w.state()


def _compare(batch, idx, ref, p):
    g = batch.read_walker(idx)
    tag = f"walker {idx} (L={p.L} ell={p.ell} seed={p.seed} w={p.walker} boundary={p.boundary})"
    assert g.stats["attempts"] == ref.attempts, tag
    assert g.stats["accepts"] == ref.accepts, tag
    assert g.stats["stages"] == ref.stages, tag
    assert g.stats["k"] == ref.k, tag
    assert g.stats["final_lnf"] == ref.lnf, tag
    ref_lng = np.where(ref.vis > 0, ref.lng, -np.inf)
    assert np.array_equal(_bits(g.lng), _bits(ref_lng)), tag
    assert np.array_equal(g.h, ref.h), tag
    assert np.array_equal(g.spins, ref.spins), tag
    assert np.array_equal(g.up.astype(np.int32), ref.up), tag


def _mixed_lines(sizes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for L in sizes:
        N = L * L
        for e in (1, 2, 3, N // 4, N // 2, N - 1, int(rng.integers(4, N - 4))):
            for bc in (1, 0):
                out.append(LineSpec(L=L, ell=e, seed=int(rng.integers(1, 2 ** 40)), walker=int(rng.integers(0, 9)),
                                    lnf0=1.0, lnf_min=float(rng.choice([1e-3, 1e-7])),
                                    flatness=float(rng.choice([0.6, 0.8])),
                                    check_interval=int(rng.choice([64, 300, 1500])),
                                    reset_checks=int(rng.choice([0, 0, 3])), boundary=bc))
    return out


@pytest.mark.parametrize("placement", [1, 2, 3, 4])
def test_open_and_periodic_bitwise(placement):
    """L = 4..64 (one word per row), open and periodic walkers side by side,
    in three chunks on each placement (the window placement keeps open
    walkers in the lattice-in-LDS form)."""
    lines = _mixed_lines((4, 6, 8, 10, 16, 34, 64), 11 + placement)
    chunks = [777, 5000, 20000]
    _say(f"open: {len(lines)} walkers, placement {placement}, chunks {chunks}")
    b = wl.Batch(lines, placement=placement, tail_walkers=-1)
    for c in chunks:
        b.advance(c)
    with ThreadPoolExecutor(8) as pool:
        refs = list(pool.map(lambda p: _oracle_state(p, sum(chunks)), lines))
    assert sum(r.stages for r, p in zip(refs, lines) if p.boundary) > 0
    for i, (p, r) in enumerate(zip(lines, refs)):
        _compare(b, i, r, p)


def test_open_wide_lattices_bitwise():
    """Device-memory kernels with two and three words per row."""
    lines = _mixed_lines((66, 130), 5)
    chunks = [1500, 12000]
    _say(f"open wide: {len(lines)} walkers, chunks {chunks}")
    b = wl.Batch(lines)
    for c in chunks:
        b.advance(c)
    with ThreadPoolExecutor(8) as pool:
        refs = list(pool.map(lambda p: _oracle_state(p, sum(chunks)), lines))
    for i, (p, r) in enumerate(zip(lines, refs)):
        _compare(b, i, r, p)


def test_open_dos_L4_assembly_thermo_and_exact():
    """All 17 open 4 x 4 lines, four walkers each (the configuration the
    oracle is pinned with), run to the end on the device with long flatness
    intervals; the device assembly equals the
    oracle's on the same lines, stays within the exact-DOS bounds of brute
    force, and its thermodynamics equal the oracle's."""
    L, N = 4, 16
    lines = [LineSpec(L=L, ell=e, seed=s, lnf_min=1e-6, check_interval=16384 * 16, boundary=1)
             for e in range(N + 1) for s in (1, 2, 3, 4)]
    _say("open 4x4 DOS: run to end")
    b = wl.Batch(lines)
    b.run_to_end()
    packed, offs = b.lng()
    W = 4
    kl, gk = wl.assemble(L, packed, N + 1, W, boundary=1)
    host = packed.cpu().numpy()
    per_line = [np.stack([host[offs[e * W + w]:offs[e * W + w + 1]] for w in range(W)]) for e in range(N + 1)]
    rkl, rgk = oracle.assemble(L, per_line, boundary=1)
    kl_h, gk_h = kl.cpu().numpy(), gk.cpu().numpy()
    assert kl_h.shape == (N + 1, 2 * L * (L - 1) + 1)
    assert np.array_equal(np.isinf(kl_h), np.isinf(rkl))
    fin = np.isfinite(rkl)
    assert np.max(np.abs(kl_h[fin] - rkl[fin])) < 1e-11
    fin = np.isfinite(rgk)
    assert np.max(np.abs(gk_h[fin] - rgk[fin])) < 1e-11
    bf = exact.brute_force(L, boundary=1)
    err = [abs(kl_h[e, k] - math.log(bf[e, k])) for e in range(N + 1) for k in range(bf.shape[1]) if bf[e, k]]
    assert np.all(np.isneginf(kl_h[bf == 0]))
    assert np.mean(err) <= 0.01 and np.max(err) <= 0.05
    beta = np.array([0.2, 0.44, 0.9, 1.3])
    H = np.array([0.0, 0.3, -0.2, 0.05])
    out, sc = wl.thermo(L, kl, beta, H, 1.0, boundary=1)
    got = out.cpu().numpy()
    for i in range(len(beta)):
        ref = thermo.thermo(L, kl_h, beta[i], H[i], 1.0, boundary=1)
        for j, f in enumerate(wl.THERMO_FIELDS):
            assert got[i, j] == pytest.approx(ref[f], rel=1e-10, abs=1e-12), (i, f)
    assert sc.item() == pytest.approx(thermo.center_entropy(L, kl_h, boundary=1), rel=1e-15)


def test_open_thermo_exact_plane():
    """wl_thermo on the exact open 4 x 4 plane against spin enumeration."""
    L = 4
    lng = thermo.lng_from_counts(exact.brute_force(L, boundary=1), boundary=1)
    dev = torch.from_numpy(np.ascontiguousarray(lng)).cuda()
    beta = np.array([0.1, 0.5, 1.2])
    H = np.array([0.4, -0.1, 0.0])
    out, _ = wl.thermo(L, dev, beta, H, 1.0, boundary=1)
    got = out.cpu().numpy()
    for i in range(len(beta)):
        ref = thermo.spin_enumeration(L, beta[i], H[i], 1.0, boundary=1)
        for j, f in enumerate(wl.THERMO_FIELDS):
            assert got[i, j] == pytest.approx(ref[f], rel=1e-10, abs=1e-12), (i, f)
