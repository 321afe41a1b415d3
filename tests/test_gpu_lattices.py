"""Triangular and honeycomb lattices on the GPU: bit-exact walker
trajectories against the oracle (periodic and open, mixed with square
walkers in one batch, on lattices of one to four words per row, on every
placement a batch can ask for: the non-square walkers run the lane kernels
with the lattice in LDS or in device memory); assembly of their lines; the
whole 4 x 4 DOS of each geometry within the exact-DOS bounds of brute
force; thermodynamics of the exact planes against spin enumeration."""
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

GEOS = [(1, 0), (1, 1), (2, 0), (2, 1)]     # (lattice, boundary)


def _say(msg):
    say(msg)


def _bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


def _oracle_state(p, attempts):
    w = oracle.Walker(p.L, p.ell, p.seed, p.walker, p.lnf0, p.lnf_min, p.flatness, p.check_interval,
                      reset_checks=p.reset_checks, boundary=p.boundary, lattice=p.lattice)
    w.advance(attempts)
    return w.state()


def _compare(batch, idx, ref, p):
    g = batch.read_walker(idx)
    tag = f"walker {idx} (L={p.L} ell={p.ell} seed={p.seed} w={p.walker} lattice={p.lattice} bc={p.boundary})"
    assert g.stats["nb"] == ref.nb == p.nb, tag
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


def _mixed_lines(sizes, seed, geos=GEOS + [(0, 0), (0, 1)]):
    rng = np.random.default_rng(seed)
    out = []
    for L in sizes:
        N = L * L
        for e in (1, 2, N // 4, N // 2, N - 1, int(rng.integers(4, N - 4))):
            for lat, bc in geos:
                out.append(LineSpec(L=L, ell=e, seed=int(rng.integers(1, 2 ** 40)), walker=int(rng.integers(0, 9)),
                                    lnf0=1.0, lnf_min=float(rng.choice([1e-3, 1e-7])),
                                    flatness=float(rng.choice([0.6, 0.8])),
                                    check_interval=int(rng.choice([64, 300, 1500])),
                                    reset_checks=int(rng.choice([0, 0, 3])), boundary=bc, lattice=lat))
    return out


@pytest.mark.parametrize("placement,wpw", [(1, 64), (1, 16), (3, 64), (2, 64), (4, 64)])
def test_lattices_bitwise(placement, wpw):
    """L = 4..64 (one word per row), every geometry side by side, in three
    chunks; placements 2 and 4 keep the non-square walkers in the
    lattice-in-LDS form."""
    lines = _mixed_lines((4, 6, 8, 12, 34, 64), 21 + placement + wpw)
    chunks = [777, 5000, 20000]
    _say(f"lattices: {len(lines)} walkers, placement {placement}, wpw {wpw}, chunks {chunks}")
    b = wl.Batch(lines, placement=placement, walkers_per_wave=wpw, tail_walkers=-1)
    for c in chunks:
        b.advance(c)
    with ThreadPoolExecutor(8) as pool:
        refs = list(pool.map(lambda p: _oracle_state(p, sum(chunks)), lines))
    assert sum(r.stages for r, p in zip(refs, lines) if p.lattice) > 0
    for i, (p, r) in enumerate(zip(lines, refs)):
        _compare(b, i, r, p)


def test_lattices_wide_bitwise():
    """Device-memory kernels with two, three and four words per row."""
    lines = _mixed_lines((66, 130, 256), 9, GEOS)
    chunks = [1500, 6000]
    _say(f"lattices wide: {len(lines)} walkers, chunks {chunks}")
    b = wl.Batch(lines)
    for c in chunks:
        b.advance(c)
    with ThreadPoolExecutor(8) as pool:
        refs = list(pool.map(lambda p: _oracle_state(p, sum(chunks)), lines))
    for i, (p, r) in enumerate(zip(lines, refs)):
        _compare(b, i, r, p)


def test_lattices_run_to_end_with_tail_switch():
    """run_to_end moves its last square walkers to one wavefront each; the
    other lattices stay on the lane kernel and still end where the oracle
    does."""
    lines = [LineSpec(L=8, ell=e, seed=3, lnf_min=1e-3, check_interval=512, lattice=lat, boundary=bc)
             for e in (5, 17, 32) for lat, bc in GEOS + [(0, 0)]]
    _say(f"lattices run to end: {len(lines)} walkers")
    b = wl.Batch(lines)
    b.run_to_end(chunk=4096)
    for i, p in enumerate(lines):
        lng, info = oracle.line_run(p.L, p.ell, p.seed, p.walker, p.lnf0, p.lnf_min, p.flatness,
                                    p.check_interval, boundary=p.boundary, lattice=p.lattice)
        g = b.read_walker(i)
        assert g.stats["done"] == 1 and g.stats["attempts"] == info.attempts, (i, p)
        assert np.array_equal(_bits(g.lng), _bits(lng)), (i, p)


def test_lattice_dos_L4_assembly_and_exact():
    """Lines 0..8 of the 4 x 4 lattice of every geometry, four walkers each,
    to the end in one batch with the flatness interval the oracle is pinned
    with; the device assembly (mirrored to ell > 8) equals the oracle's on
    the same lines and lies within mean 0.01 / max 0.05 of brute force."""
    L, N, W = 4, 16, 4
    lines = [LineSpec(L=L, ell=e, seed=s, lnf_min=1e-6, check_interval=1 << 20, boundary=bc, lattice=lat)
             for lat, bc in GEOS for e in range(N // 2 + 1) for s in range(1, W + 1)]
    _say(f"lattice 4x4 DOS: {len(lines)} walkers to the end")
    b = wl.Batch(lines)
    b.run_to_end()
    packed, offs = b.lng()
    per = (N // 2 + 1) * W
    for gi, (lat, bc) in enumerate(GEOS):
        base = gi * per
        seg = packed[int(offs[base]):int(offs[base + per])].contiguous()
        kl, gk = wl.assemble(L, seg, N // 2 + 1, W, boundary=bc, lattice=lat)
        host = seg.cpu().numpy()
        o = offs[base:base + per + 1] - offs[base]
        per_line = [np.stack([host[o[e * W + w]:o[e * W + w + 1]] for w in range(W)]) for e in range(N // 2 + 1)]
        rkl, rgk = oracle.assemble(L, per_line, boundary=bc, lattice=lat)
        kl_h, gk_h = kl.cpu().numpy(), gk.cpu().numpy()
        tag = f"lattice {lat} boundary {bc}"
        assert kl_h.shape == rkl.shape == (N + 1, wl.n_columns(L, bc, lat)), tag
        assert np.array_equal(np.isinf(kl_h), np.isinf(rkl)), tag
        fin = np.isfinite(rkl)
        assert np.max(np.abs(kl_h[fin] - rkl[fin])) < 1e-11, tag
        fin = np.isfinite(rgk)
        assert np.max(np.abs(gk_h[fin] - rgk[fin])) < 1e-11, tag
        ref = thermo.lng_from_counts(exact.brute_force(L, bc, lat), bc, lat)
        sup = np.isfinite(ref)
        assert np.array_equal(np.isfinite(kl_h), sup), tag
        err = np.abs(kl_h[sup] - ref[sup])
        assert err.mean() <= 0.01 and err.max() <= 0.05, (tag, err.mean(), err.max())
        beta = np.array([0.2, 0.7])
        H = np.array([0.1, -0.3])
        out, sc = wl.thermo(L, kl, beta, H, 1.0, boundary=bc, lattice=lat)
        got = out.cpu().numpy()
        for i in range(len(beta)):
            r = thermo.thermo(L, kl_h, beta[i], H[i], 1.0, boundary=bc, lattice=lat)
            for j, f in enumerate(wl.THERMO_FIELDS):
                assert got[i, j] == pytest.approx(r[f], rel=1e-10, abs=1e-12), (tag, i, f)
        assert sc.item() == pytest.approx(thermo.center_entropy(L, kl_h, bc, lat), rel=1e-15), tag


@pytest.mark.parametrize("lattice,boundary", GEOS)
def test_lattice_thermo_exact_plane(lattice, boundary):
    """wl_thermo_ex on the exact 4 x 4 plane against spin enumeration."""
    L = 4
    lng = thermo.lng_from_counts(exact.brute_force(L, boundary, lattice), boundary, lattice)
    dev = torch.from_numpy(np.ascontiguousarray(lng)).cuda()
    beta = np.array([0.1, 0.5, 1.2])
    H = np.array([0.4, -0.1, 0.0])
    for J in (1.0, -1.0):
        out, _ = wl.thermo(L, dev, beta, H, J, boundary=boundary, lattice=lattice)
        got = out.cpu().numpy()
        for i in range(len(beta)):
            ref = thermo.spin_enumeration(L, beta[i], H[i], J, boundary=boundary, lattice=lattice)
            for j, f in enumerate(wl.THERMO_FIELDS):
                assert got[i, j] == pytest.approx(ref[f], rel=1e-10, abs=1e-12), (J, i, f)
