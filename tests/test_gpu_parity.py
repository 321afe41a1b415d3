"""GPU library vs the CPU oracle, walker by walker, bit for bit.

Each test runs walkers through the C ABI (wl_batch_*, wl_line_run,
wl_assemble) and the same walkers through the oracle for the same number of
proposals, then compares the complete state: counters, k, ln f, the spin
configuration, both site lists, ln g (as bit patterns, -inf where never
visited) and the histogram.
"""
import math
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


def _oracle_state(p, attempts):
    w = oracle.Walker(p.L, p.ell, p.seed, p.walker, p.lnf0, p.lnf_min, p.flatness, p.check_interval,
                      reset_checks=getattr(p, "reset_checks", 0), boundary=getattr(p, "boundary", 0))
    w.advance(attempts)
    return w.state()


def _oracle_states(lines, attempts):
    with ThreadPoolExecutor(8) as pool:
        return list(pool.map(lambda p: _oracle_state(p, attempts), lines))


def _bits(x):
    return np.asarray(x, dtype=np.float64).view(np.uint64)


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
    ref_lng = np.where(ref.vis > 0, ref.lng, -np.inf)
    assert np.array_equal(_bits(g.lng), _bits(ref_lng)), tag
    assert np.array_equal(g.h, ref.h), tag
    assert np.array_equal(g.spins, ref.spins), tag
    assert np.array_equal(g.up.astype(np.int32), ref.up), tag
    assert np.array_equal(g.dn.astype(np.int32), ref.dn), tag


@pytest.mark.parametrize("tail", [0, -1])
def test_c1_full_run_bitwise(tail):
    """tail 0: the 17 walkers run with one wavefront each (placement 4) from
    the first chunk; tail -1: lane-per-walker throughout."""
    lines = workloads.c1()
    _say(f"c1: {len(lines)} walkers to completion, tail_walkers {tail}")
    b = wl.Batch(lines, tail_walkers=tail)
    b.run_to_end(chunk=1 << 16)
    refs = _oracle_states(lines, (1 << 64) - 1)
    for i, (p, r) in enumerate(zip(lines, refs)):
        assert r.done
        _compare(b, i, r, p)
    # packed output agrees with the per-walker read-back
    for i, arr in enumerate(b.lng_list()):
        assert np.array_equal(_bits(arr), _bits(np.where(refs[i].vis > 0, refs[i].lng, -np.inf)))


def _mixed_lines():
    out = []
    rng = np.random.default_rng(2024)
    for L in (4, 6, 8, 10, 12, 16, 24, 32, 48, 64):
        N = L * L
        ells = sorted(set([0, 1, 2, N // 2, N - 1, N] + [int(x) for x in rng.integers(0, N + 1, 4)]))
        for e in ells:
            out.append(LineSpec(L=L, ell=e, seed=int(rng.integers(1, 2 ** 40)), walker=int(rng.integers(0, 9)),
                                lnf0=1.0, lnf_min=float(rng.choice([1e-3, 1e-6, 1e-8])),
                                flatness=float(rng.choice([0.6, 0.8, 0.95])),
                                check_interval=int(rng.choice([0, 100, 999, 4 * N]))))
    return out


@pytest.mark.parametrize("wpw,placement", [(0, 0), (16, 1), (32, 1), (64, 1), (64, 2), (64, 3), (16, 3), (0, 4),
                                         (0, 5), (0, 6), (0, 7), (0, 8)])
def test_mixed_batch_chunked_bitwise(wpw, placement):
    """Every launch variant (placement of the hot state, walkers per
    wavefront) walks the same trajectories."""
    lines = _mixed_lines()
    chunks = [777, 4096, 20000]
    _say(f"mixed: {len(lines)} walkers, {wpw} per wavefront, placement {placement}, chunks {chunks}")
    b = wl.Batch(lines, walkers_per_wave=wpw, placement=placement)
    for c in chunks:
        b.advance(c)
    refs = _oracle_states(lines, sum(chunks))
    for i, (p, r) in enumerate(zip(lines, refs)):
        _compare(b, i, r, p)


@pytest.mark.parametrize("L,placement", [(32, 5), (32, 6), (32, 7), (16, 7), (8, 7), (64, 8), (32, 8), (16, 8),
                                         (8, 8), (6, 8)])
def test_uniform_side_chunked_bitwise(L, placement):
    """A batch whose walkers all have one L takes the kernels specialised for
    that side (L = 32: wraps by mask); short check intervals take the narrow
    lines through flatness tests, stage transitions and completion."""
    N = L * L
    rng = np.random.default_rng(L * 10 + placement)
    ells = sorted(set([1, 2, 3, N // 2, N // 2 - 1, N - 1] + [int(x) for x in rng.integers(4, N - 4, 10)]))
    lines = [LineSpec(L=L, ell=e, seed=int(rng.integers(1, 2 ** 40)), walker=int(rng.integers(0, 9)),
                      lnf_min=float(rng.choice([1e-2, 1e-4])), check_interval=int(rng.choice([64, 300, 2 * N])))
             for e in ells]
    chunks = [777, 4096, 30000]
    _say(f"uniform L={L}: {len(lines)} walkers, placement {placement}, chunks {chunks}")
    b = wl.Batch(lines, placement=placement)
    for c in chunks:
        b.advance(c)
    refs = _oracle_states(lines, sum(chunks))
    assert any(r.done for r in refs) and any(r.stages > 0 and not r.done for r in refs)
    for i, (p, r) in enumerate(zip(lines, refs)):
        _compare(b, i, r, p)


def test_c2_prefix_bitwise():
    lines = workloads.c2()
    T = 1 << 19
    _say(f"c2: {len(lines)} walkers, {T} attempts")
    b = wl.Batch(lines)
    b.advance(T)
    refs = _oracle_states(lines, T)
    for i, (p, r) in enumerate(zip(lines, refs)):
        _compare(b, i, r, p)


def test_c2_lines_to_completion_bitwise():
    """Lane-per-walker until at most 5 walkers are left, then one wavefront
    each (the switch happens between chunks, mid-run)."""
    lines = [p for p in workloads.c2() if p.ell in (1, 2, 5, 31, 63) and p.seed in (1, 3)]
    _say(f"c2 lines to completion: {len(lines)} walkers")
    b = wl.Batch(lines, tail_walkers=5)
    chunks = 0
    while b.run(1 << 16, 1) > 0:
        chunks += 1
    refs = _oracle_states(lines, (1 << 64) - 1)
    for i, (p, r) in enumerate(zip(lines, refs)):
        assert r.done
        _compare(b, i, r, p)


@pytest.mark.parametrize("placement", [0, 1, 2, 5, 6, 7, 8])
def test_l64_workload_sampled_bitwise(placement):
    """The attempts/s workload (64x64, 2049 lines x 8 walkers) in the launch
    configuration the benchmark times; sampled walkers checked against the oracle."""
    lines = workloads.l64()
    S = 1 << 16
    _say(f"l64: {len(lines)} walkers, placement {placement}, one launch of {S} attempts")
    b = wl.Batch(lines, placement=placement)
    b.advance(S)
    rng = np.random.default_rng(7)
    idx = sorted(set([0, 1, 2, 8 * 2048, 8 * 2048 + 7, 8 * 1024 + 3] +
                     [int(x) for x in rng.integers(0, len(lines), 40)]))
    refs = _oracle_states([lines[i] for i in idx], S)
    for i, r in zip(idx, refs):
        _compare(b, i, r, lines[i])
    st = b.stats()
    # every walker on a line with moves made exactly S proposals (no line can
    # finish 14 stages within S = 16N attempts); lines 0 and N make none
    ells = np.array([p.ell for p in lines])
    expect = np.where((ells == 0) | (ells == 4096), 0, S)
    assert np.array_equal(st["attempts"].astype(np.int64), expect)


def test_pc_kernel_workspace_beyond_4gib_bitwise():
    """The producer/consumer kernel addresses the walker arrays by 32-bit
    offsets while the workspace spans less than 4 GiB and by full addresses
    beyond: the L = 64 lines with 64 walkers each (131136 walkers, 5.5 GB)
    take the second form; sampled walkers against the oracle."""
    lines = workloads.l64(64)
    S = 1 << 12
    _say(f"l64 x 32: {len(lines)} walkers, placement 6, two launches of {S} attempts")
    b = wl.Batch(lines, placement=6)
    assert b.ws_bytes > (1 << 32)
    b.advance(S)
    b.advance(S)
    rng = np.random.default_rng(41)
    idx = sorted(set([0, 1, 63, 64 * 2048, len(lines) - 1] + [int(x) for x in rng.integers(0, len(lines), 24)]))
    refs = _oracle_states([lines[i] for i in idx], 2 * S)
    for i, r in zip(idx, refs):
        _compare(b, i, r, lines[i])
    b.close()


def test_server_on_producer_placement_matches_oracle():
    """The job server with placement 6 (its walkers in the server's own
    arena, the kernel's full-address form) against the oracle's lines."""
    L, W, seed, lnf_min = 4, 2, 5, 1e-4
    N = L * L
    s = wl.Server(16 << 20, placement=6, tail_walkers=-1)
    try:
        jid = s.submit(L=L, W=W, seed=seed, lnf_min=lnf_min)
        s.wait(jid, 300.0)
        got = s.fetch(jid)
    finally:
        s.close()
    lines = []
    for ell in range(N // 2 + 1):
        lines.append(np.stack([oracle.line_run(L, ell, seed, walker=w, lnf_min=lnf_min)[0] for w in range(W)]))
    ref, _ = oracle.assemble(L, lines, n_lines=N // 2 + 1)
    assert np.array_equal(np.isinf(got), np.isinf(ref))
    fin = np.isfinite(ref)
    assert np.max(np.abs(got[fin] - ref[fin])) < 1e-11


def _reset_lines():
    """Lines with extra resets at unchanged f (reset_checks 1..5), including
    flatness 1.0 (every test fails, so every reset_checks-th test resets)."""
    out = []
    rng = np.random.default_rng(31)
    for L in (4, 6, 8, 12, 16, 32, 64, 66, 128):
        N = L * L
        for e in (1, 3, N // 2, int(rng.integers(4, N - 4))):
            out.append(LineSpec(L=L, ell=e, seed=int(rng.integers(1, 2 ** 40)), walker=int(rng.integers(0, 9)),
                                lnf0=1.0, lnf_min=float(rng.choice([1e-3, 1e-6])),
                                flatness=float(rng.choice([0.8, 1.0])),
                                check_interval=int(rng.choice([64, 300])),
                                reset_checks=int(rng.choice([1, 2, 5]))))
    return out


@pytest.mark.parametrize("placement", [1, 2, 3, 4, 5, 6, 7, 8])
def test_extra_resets_bitwise(placement):
    """Extra resets at unchanged f walk the oracle's trajectories in every
    kernel (lane with the lattice in LDS, with the ln g window, all in device
    memory, one wavefront per walker; L > 64 on the device-memory kernel)."""
    lines = _reset_lines()
    chunks = [999, 7000, 25000]
    _say(f"resets: {len(lines)} walkers, placement {placement}, chunks {chunks}")
    b = wl.Batch(lines, placement=placement, tail_walkers=-1)
    for c in chunks:
        b.advance(c)
    refs = _oracle_states(lines, sum(chunks))
    assert sum(r.stages for r in refs) > 0
    for i, (p, r) in enumerate(zip(lines, refs)):
        _compare(b, i, r, p)


def _wide_lines():
    out = []
    rng = np.random.default_rng(77)
    for L in (66, 96, 128, 130, 194, 256):
        N = L * L
        for e in (1, 2, N // 3, N // 2, N - 1, int(rng.integers(3, N - 3))):
            out.append(LineSpec(L=L, ell=e, seed=int(rng.integers(1, 2 ** 40)), walker=int(rng.integers(0, 9)),
                                lnf0=1.0, lnf_min=float(rng.choice([1e-2, 1e-8])),
                                flatness=float(rng.choice([0.5, 0.8])),
                                check_interval=int(rng.choice([64, 333, 2000]))))
    return out


@pytest.mark.parametrize("wpw,wide", [(0, 0), (16, 0), (32, 0), (0, 1)])
def test_wide_lattices_chunked_bitwise(wpw, wide):
    """Lattices wider than one 64-bit word per row (L = 66..256: kernels with
    2..4 words per row, the lattice in device memory or, wide = 1, in LDS),
    short flatness intervals so that stage transitions happen inside the
    window."""
    lines = _wide_lines()
    chunks = [1001, 9000, 30000]
    _say(f"wide: {len(lines)} walkers, {wpw} per wavefront, wide placement {wide}, chunks {chunks}")
    b = wl.Batch(lines, walkers_per_wave=wpw, wide_placement=wide)
    for c in chunks:
        b.advance(c)
    refs = _oracle_states(lines, sum(chunks))
    assert any(r.stages > 0 for r in refs)
    for i, (p, r) in enumerate(zip(lines, refs)):
        _compare(b, i, r, p)


def _sampled_window(lines, launches, attempts, n_sample, seed, must=()):
    b = wl.Batch(lines)
    for _ in range(launches):
        b.advance(attempts)
    rng = np.random.default_rng(seed)
    idx = sorted(set(list(must) + [int(x) for x in rng.integers(0, len(lines), n_sample)]))
    refs = _oracle_states([lines[i] for i in idx], launches * attempts)
    for i, r in zip(idx, refs):
        _compare(b, i, r, lines[i])
    return b


def test_c3_workload_sampled_bitwise():
    """32x32, lines 0..512 x 8 walkers, in the benchmark's launch
    configuration (launches of 16384 proposals)."""
    lines = workloads.c3()
    _say(f"c3: {len(lines)} walkers, 2 launches of 16384")
    b = _sampled_window(lines, 2, 16384, 40, 11, must=(0, 8, 8 * 512, 8 * 512 + 7, 8 * 256))
    b.close()


def test_c5_workload_sampled_bitwise():
    """256x256, lines 0..32768, one walker each (21.8 GB of walker state), in
    the benchmark's launch configuration (launches of 16384 proposals)."""
    lines = workloads.c5()
    _say(f"c5: {len(lines)} walkers, 2 launches of 16384")
    b = _sampled_window(lines, 2, 16384, 24, 13, must=(0, 1, 2, 16384, 32767, 32768))
    b.close()


def test_batch_run_counts_and_matches_run_to_end():
    """wl_batch_run returns the number of walkers still walking (as the stats
    show) and, chunk by chunk with the tail switch, ends in the same state as
    wl_batch_run_to_end on lane-per-walker kernels only."""
    lines = [LineSpec(L=6, ell=e, seed=9, walker=w, lnf_min=1e-4) for e in range(0, 37) for w in range(2)]
    _say(f"batch run: {len(lines)} walkers")
    a = wl.Batch(lines, tail_walkers=20)
    counts = []
    while True:
        active = a.run(1 << 12, 1)
        st = a.stats()
        assert active == int((st["done"] == 0).sum())
        counts.append(active)
        if active == 0:
            break
    assert counts == sorted(counts, reverse=True) and counts[-1] == 0
    b = wl.Batch(lines, tail_walkers=-1)
    b.run_to_end(chunk=1 << 12)
    for i in range(len(lines)):
        ga, gb = a.read_walker(i), b.read_walker(i)
        assert ga.stats == gb.stats, i
        assert np.array_equal(_bits(ga.lng), _bits(gb.lng)), i
        assert np.array_equal(ga.h, gb.h) and np.array_equal(ga.spins, gb.spins), i


@pytest.mark.parametrize("lo,hi", [(-80.0, 0.0), (-1.0, 0.0), (-1e-3, 0.0), (-80.0, -60.0)])
def test_accept_estimate_within_margin(lo, hi):
    """The single-precision estimate behind the acceptance shortcut stays far
    inside its 2^-14 margin (so every decision equals u < exp_fixed(D))."""
    err = wl.selfcheck_accept(lo, hi, 1 << 24)
    _say(f"accept estimate on [{lo}, {hi}]: max relative error {err:.3e}")
    assert 0.0 <= err < 2.0 ** -17


@pytest.mark.parametrize("lo,hi", [(-800.0, -1e-12), (-40.0, -1e-12), (-1e-3, -1e-15), (-800.0, -700.0)])
def test_log_bounds_settle_like_the_plain_test(lo, hi):
    """The ln u bounds of the one-wavefront-per-walker kernel never settle an
    acceptance test differently from u < exp_fixed(D), with u at, next to and
    around exp_fixed(D) and spread over [0, 1)."""
    n = 1 << 18
    settled, wrong = wl.selfcheck_threshold(lo, hi, n)
    _say(f"ln u bounds on [{lo}, {hi}]: {settled} settled, {wrong} wrong")
    assert wrong == 0
    assert settled >= 20 * n


def test_line_run_host_api():
    for ell in (0, 1, 3, 8, 12, 16):
        got, gst = wl.line_run(4, ell, 1, 1.0, 1e-6, 0.8)
        ref, rinfo = oracle.line_run(4, ell, 1, lnf_min=1e-6)
        assert np.array_equal(_bits(got), _bits(ref)), ell
        assert gst["attempts"] == rinfo.attempts and gst["stages"] == rinfo.stages
    p = LineSpec(L=6, ell=11, seed=5, walker=2, lnf0=1.0, lnf_min=1e-5, flatness=0.8, check_interval=500)
    got, _ = wl.line_run_ex(p)
    ref, _ = oracle.line_run(6, 11, 5, walker=2, lnf_min=1e-5, check_interval=500)
    assert np.array_equal(_bits(got), _bits(ref))


def test_assemble_matches_oracle():
    import torch
    for L, n_lines, W, seeds in ((4, 17, 1, [1]), (4, 9, 2, [1, 2])):
        N = L * L
        lines = [LineSpec(L=L, ell=e, seed=s, lnf_min=1e-6) for e in range(n_lines) for s in seeds]
        b = wl.Batch(lines)
        b.run_to_end()
        packed, offs = b.lng()
        kl, gk = wl.assemble(L, packed, n_lines, W)
        host = packed.cpu().numpy()
        per_line = [np.stack([host[offs[e * W + w]:offs[e * W + w + 1]] for w in range(W)])
                    for e in range(n_lines)]
        rkl, rgk = oracle.assemble(L, per_line, n_lines=n_lines)
        kl, gk = kl.cpu().numpy(), gk.cpu().numpy()
        assert np.array_equal(np.isinf(kl), np.isinf(rkl))
        fin = np.isfinite(rkl)
        assert np.max(np.abs(kl[fin] - rkl[fin])) < 1e-11
        fin = np.isfinite(rgk)
        assert np.array_equal(np.isinf(gk), np.isinf(rgk))
        assert np.max(np.abs(gk[fin] - rgk[fin])) < 1e-11
        # Eq. 4 holds per line after assembly
        for e in range(N + 1):
            row = kl[e][np.isfinite(kl[e])]
            mx = row.max()
            assert abs(mx + math.log(np.exp(row - mx).sum()) - oracle.log_binomial(N, e)) < 1e-10


def test_run_async_matches_run_to_end():
    """wl_batch_run_async (enqueue only, one launch per class to the end)
    leaves every walker where wl_batch_run_to_end does (without its switch to
    one wavefront per walker): packed ln g bit for bit, same counters."""
    import torch
    lines = [LineSpec(L=L, ell=e, seed=5, walker=w, lnf_min=1e-4)
             for L in (4, 6, 8) for e in range(0, L * L + 1, 3) for w in range(2)]
    _say(f"run_async: {len(lines)} walkers")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        lng, offs, stats, ws = wl.run_async(lines, stream=stream)
    ev = torch.cuda.Event()
    ev.record(stream)
    ev.synchronize()
    got = lng.cpu().numpy()
    st = np.frombuffer(stats.cpu().numpy().tobytes(), dtype=wl.STATS_DTYPE)
    b = wl.Batch(lines, tail_walkers=-1)
    b.run_to_end(chunk=1 << 14)
    ref = b.lng_list()
    rst = b.stats()
    for i in range(len(lines)):
        assert np.array_equal(_bits(got[offs[i]:offs[i + 1]]), _bits(ref[i])), i
    assert np.array_equal(st["attempts"], rst["attempts"]) and np.array_equal(st["done"], rst["done"])
    assert (st["done"] == 1).all()


def test_tuned_check_interval_is_the_tables():
    """check_interval = WL_CHECK_INTERVAL_TUNED walks exactly as the explicit
    interval factor(L) * N from the autotuner's table (so any other
    implementation reproduces it from the table)."""
    from paper_1302_2320_amd import autotune
    tuned = (1 << 64) - 1
    base = [LineSpec(L=L, ell=e, seed=3, lnf_min=1e-3) for L in (6, 8, 16) for e in (2, L * L // 3)]
    a = wl.Batch([LineSpec(**{**p.__dict__, "check_interval": tuned}) for p in base])
    b = wl.Batch([LineSpec(**{**p.__dict__, "check_interval": autotune.check_factor_for(p.L) * p.L * p.L})
                  for p in base])
    for x in (a, b):
        x.advance(300000)
    for i in range(len(base)):
        ga, gb = a.read_walker(i), b.read_walker(i)
        assert ga.stats == gb.stats, i
        assert np.array_equal(_bits(ga.lng), _bits(gb.lng)), i
