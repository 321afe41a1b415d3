"""wl_thermo_noalloc (static device scratch, no allocation) against
wl_thermo_ex (stream-ordered scratch): the same kernels in the same order, so
the results must agree bit for bit, on two calls in a row, the second one
smaller (the static buffer keeps the first call's contents).  Named to be
collected last, after the other GPU tests."""
import ctypes
import sys

import numpy as np
import pytest

from paper_1302_2320_amd import wl

pytestmark = pytest.mark.gpu


def _plane(L, seed):
    """A smooth synthetic ln g(k, ell) plane with the support of the periodic
    square lattice (row ell, column q <-> k = 2q), -inf outside it."""
    N = L * L
    rng = np.random.default_rng(seed)
    ell = np.arange(N + 1)[:, None]
    q = np.arange(N + 1)[None, :]
    m = np.minimum(ell, N - ell)
    lng = np.where(q <= 2 * m, 0.5 * N * (1.0 - ((q - m) / (m + 1.0)) ** 2), -np.inf)
    return lng + np.where(np.isfinite(lng), rng.normal(0.0, 0.3, lng.shape), 0.0)


def _call(fn, L, plane, beta, H, J=1.0):
    import torch
    out = torch.empty((beta.numel(), 6), dtype=torch.float64, device="cuda")
    sc = torch.empty(1, dtype=torch.float64, device="cuda")
    st = fn(L, 0, 0, ctypes.c_void_p(plane.data_ptr()), J, beta.numel(), ctypes.c_void_p(beta.data_ptr()),
            ctypes.c_void_p(H.data_ptr()), ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(sc.data_ptr()),
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == wl.WL_OK, wl.lib().wl_last_error()
    torch.cuda.synchronize()
    return out.cpu().numpy(), sc.cpu().numpy()


def test_noalloc_equals_thermo_on_two_calls():
    import torch
    lib = wl.lib()
    for L, npts, seed in ((32, 256, 1), (16, 37, 2)):       # second call smaller
        print(f"noalloc: L={L}, {npts} points", flush=True)
        sys.stdout.flush()
        plane = torch.from_numpy(_plane(L, seed)).cuda()
        beta = torch.linspace(0.05, 1.2, npts, dtype=torch.float64, device="cuda")
        H = torch.linspace(-0.7, 0.4, npts, dtype=torch.float64, device="cuda")
        a, sa = _call(lib.wl_thermo_noalloc, L, plane, beta, H)
        b, sb = _call(lib.wl_thermo_ex, L, plane, beta, H)
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
        assert np.array_equal(sa.view(np.uint64), sb.view(np.uint64))
        assert np.isfinite(a).all()


def test_noalloc_rejects_beyond_its_buffer():
    import torch
    L, npts = 32, 4096                      # 4096 points * 7 doubles * (>= 2 chunks) > 2^20
    plane = torch.from_numpy(_plane(L, 3)).cuda()
    beta = torch.full((npts,), 0.4, dtype=torch.float64, device="cuda")
    H = torch.zeros(npts, dtype=torch.float64, device="cuda")
    out = torch.empty((npts, 6), dtype=torch.float64, device="cuda")
    st = wl.lib().wl_thermo_noalloc(L, 0, 0, ctypes.c_void_p(plane.data_ptr()), 1.0, npts,
                                    ctypes.c_void_p(beta.data_ptr()), ctypes.c_void_p(H.data_ptr()),
                                    ctypes.c_void_p(out.data_ptr()), None, None)
    assert st == wl.WL_EINVAL
    assert b"at most" in wl.lib().wl_last_error()
