"""The arithmetic shortcuts of the one-wavefront walks, checked as claims on
random doubles (host only; the kernels' use of them is checked bit for bit
by the GPU parity tests).

- Closed-form growth: when ln f is a power of two, cur < 2^53 ln f and
  cur + n ln f stays in cur's binade, adding ln f n times (each addition
  rounded) gives exactly cur + n ln f; across a binade the shortcut would
  be wrong, which is why the kernels test for it.
- Certain decisions: with Rl = ((g' + lo) - slack) - (s - last) ln f (1 +
  2^-40) and Al = min(g', (g' + hi) + slack), slack = 2^-20 + 2^-40 |g'|, a
  lane whose current ln g is below Rl still has D = cur' - g' < lo after up
  to s - last additions of ln f (cur' the grown value), and a lane at or
  above Al has D >= 0 or D > hi; lo and hi are the bounds the acceptance
  test takes as certain.
"""
import numpy as np


def _add_seq(cur, lnf, n):
    for _ in range(n):
        cur = cur + lnf
    return cur


def _closed_form_applies(cur, lnf, n):
    b = np.float64(lnf).view(np.uint64)
    pow2 = (int(b) & 0x000FFFFFFFFFFFFF) == 0 and (int(b) >> 52) != 0
    cn = cur + float(n) * lnf
    hc = int(np.float64(cur).view(np.uint64)) >> 32
    hn = int(np.float64(cn).view(np.uint64)) >> 32
    return pow2 and cur < lnf * 2.0 ** 53 and (hc ^ hn) < 0x00100000, cn


def test_closed_form_growth_equals_repeated_additions():
    rng = np.random.default_rng(1)
    hits = 0
    for _ in range(20000):
        lnf = 2.0 ** -int(rng.integers(0, 40))
        cur = float(rng.uniform(0.0, 1.0)) * 2.0 ** int(rng.integers(-5, 25))
        n = int(rng.integers(1, 65))
        ok, cn = _closed_form_applies(cur, lnf, n)
        if ok:
            hits += 1
            assert cn == _add_seq(cur, lnf, n), (cur, lnf, n)
    assert hits > 5000


def test_closed_form_would_fail_across_a_binade():
    # an odd multiple of the ulp just below 2: the sum leaves the binade and
    # the one-shot value differs from the repeated additions
    cur = 2.0 - 2.0 ** -52
    lnf = 2.0 ** -51
    ok, cn = _closed_form_applies(cur, lnf, 2)
    assert not ok
    assert cn != _add_seq(cur, lnf, 2)


def test_certain_decisions_hold_after_the_growth():
    rng = np.random.default_rng(2)
    checked_rej = checked_acc = 0
    for _ in range(40000):
        lnf = 2.0 ** -int(rng.integers(0, 30))
        g = float(rng.uniform(0.0, 2.0 ** int(rng.integers(0, 12))))          # ln g of the target
        lu = float(np.log(rng.uniform(2.0 ** -60, 1.0)))                       # ln u (its estimate)
        lo, hi = lu - 2.0 ** -10, lu + 2.0 ** -10
        waits = int(rng.integers(0, 65))                                        # lanes since the last decided one
        slack = 2.0 ** -20 + 2.0 ** -40 * abs(g)
        Rl = ((g + lo) - slack) - waits * (lnf * (1.0 + 2.0 ** -40))
        Al = min(g, (g + hi) + slack)
        # a current ln g near either threshold
        for cur in (np.nextafter(Rl, -np.inf), Rl - float(rng.uniform(0, 1e-3)), Al,
                    Al + float(rng.uniform(0, 1e-3))):
            cur = float(cur)
            if cur < 0.0:
                continue
            if cur < Rl:
                grown = _add_seq(cur, lnf, waits)
                assert grown - g < lo, (cur, g, lo, lnf, waits)
                checked_rej += 1
            if cur >= Al:
                D = cur - g
                assert D >= 0.0 or D > hi, (cur, g, hi)
                checked_acc += 1
    assert checked_rej > 10000 and checked_acc > 10000
