"""GPU thermodynamics (wl_thermo) against the oracle's plain evaluation of
Eq. 2: exact degeneracies (brute force at 4 x 4, transfer matrix at 6 x 6 and
8 x 8), synthetic planes at 16 x 16 and 32 x 32 (many row chunks, ragged
tails, unsupported chunks), a ragged number of points, and the whole chain
line walks -> assembly -> thermodynamics at 4 x 4."""
import sys

import numpy as np
import pytest

from _progress import say

from oracle import exact, thermo
from paper_1302_2320_amd import wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    say(msg)


def _points(n, seed):
    rng = np.random.default_rng(seed)
    beta = np.concatenate([[0.0, 0.44, 1.0], rng.uniform(0.05, 2.0, n - 3)])
    H = np.concatenate([[0.3, 0.0, -0.7], rng.uniform(-1.5, 1.5, n - 3)])
    return beta, H


def _compare(L, lng, beta, H, J, rel):
    dev = torch.from_numpy(np.ascontiguousarray(lng)).cuda()
    out, sc = wl.thermo(L, dev, beta, H, J)
    got = out.cpu().numpy()
    for i in range(len(beta)):
        ref = thermo.thermo(L, lng, beta[i], H[i], J)
        for j, f in enumerate(wl.THERMO_FIELDS):
            assert got[i, j] == pytest.approx(ref[f], rel=rel, abs=rel * 1e-2), (L, i, f)
    assert sc.item() == pytest.approx(thermo.center_entropy(L, lng), rel=1e-15)


@pytest.mark.parametrize("L", [4, 6, 8])
@pytest.mark.parametrize("J", [1.0, -1.0, 0.0])
def test_exact_planes(L, J):
    g = exact.brute_force(4) if L == 4 else np.asarray(exact.transfer_matrix(L), dtype=np.int64)
    lng = thermo.lng_from_counts(g)
    beta, H = _points(9, L)
    _say(f"thermo: exact plane L={L} J={J}, {len(beta)} points")
    _compare(L, lng, beta, H, J, 1e-10)


@pytest.mark.parametrize("L,n", [(16, 7), (32, 5), (32, 1)])
def test_synthetic_planes(L, n):
    """ln g over each line's support k <= 4 min(ell, N - ell): a smooth
    surface of the right scale plus noise; some rows empty (whole chunks
    unsupported)."""
    rng = np.random.default_rng(L * 100 + n)
    N = L * L
    lng = np.full((N + 1, N + 1), -np.inf)
    for ell in range(N + 1):
        m = min(ell, N - ell)
        if ell % 7 == 3:
            continue                                  # an empty row
        qs = np.arange(0, 2 * m + 1)
        lng[ell, qs] = 0.5 * N * (1.0 - ((qs - m) / (m + 1.0)) ** 2) + rng.normal(0.0, 0.5, qs.size)
    beta, H = _points(max(n, 3), L)
    beta, H = beta[:n], H[:n]
    _say(f"thermo: synthetic plane L={L}, {n} points")
    _compare(L, lng, beta, H, 1.0, 1e-9)


def test_chain_from_line_walks():
    """Lines run on the device, assembled on the device, thermodynamics on
    the device, against the oracle's lines, assembly and thermodynamics."""
    import oracle
    L, N = 4, 16
    lines, refs = [], []
    for ell in range(N // 2 + 1):
        got, _ = wl.line_run(L, ell, 7, 1.0, 1e-6, 0.8)
        ref, _ = oracle.line_run(L, ell, 7, lnf_min=1e-6)
        lines.append(got)
        refs.append(ref)
    packed = torch.from_numpy(np.concatenate(lines)).cuda()
    kl, _ = wl.assemble(L, packed, N // 2 + 1, 1)
    ref_kl = oracle.assemble(L, refs)[0]
    beta, H = _points(6, 3)
    out, sc = wl.thermo(L, kl, beta, H, 1.0)
    got = out.cpu().numpy()
    _say(f"thermo: chain L={L}")
    for i in range(len(beta)):
        ref = thermo.thermo(L, np.asarray(ref_kl), beta[i], H[i], 1.0)
        for j, f in enumerate(wl.THERMO_FIELDS):
            assert got[i, j] == pytest.approx(ref[f], rel=1e-9, abs=1e-11), (i, f)
