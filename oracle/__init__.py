"""CPU oracle for the micromagnetic-ensemble Wang-Landau walk.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow CPU definition the
GPU library is checked against (``wlref.c`` through ctypes) plus the exact
references that pin it (``exact.py``).  Only the tests, the smoke check and
the benchmark's cpu_baseline leg may import it; the product never does, and
nothing here imports the product.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


class WlrefParams(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("ell", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("walker", ctypes.c_uint32), ("reset_checks", ctypes.c_uint32),
                ("lnf0", ctypes.c_double), ("lnf_min", ctypes.c_double),
                ("flatness", ctypes.c_double), ("check_interval", ctypes.c_uint64),
                ("boundary", ctypes.c_uint32), ("lattice", ctypes.c_uint32)]


class WlrefInfo(ctypes.Structure):
    _fields_ = [("attempts", ctypes.c_uint64), ("accepts", ctypes.c_uint64),
                ("stages", ctypes.c_uint32), ("done", ctypes.c_uint32),
                ("k", ctypes.c_int32), ("nb", ctypes.c_int32), ("nprev", ctypes.c_int32),
                ("nfail", ctypes.c_int32), ("lnf", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        L.wlref_philox4x32_10.argtypes = [P(ctypes.c_uint32), P(ctypes.c_uint32), P(ctypes.c_uint32)]
        L.wlref_philox4x32_10.restype = None
        L.wlref_exp_fixed.argtypes = [ctypes.c_double]
        L.wlref_exp_fixed.restype = ctypes.c_double
        L.wlref_count_k.argtypes = [ctypes.c_int, P(ctypes.c_uint8)]
        L.wlref_count_k.restype = ctypes.c_int
        L.wlref_count_k_bc.argtypes = [ctypes.c_int, ctypes.c_int, P(ctypes.c_uint8)]
        L.wlref_count_k_bc.restype = ctypes.c_int
        L.wlref_count_k_geo.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_uint8)]
        L.wlref_count_k_geo.restype = ctypes.c_int
        L.wlref_n_bonds.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.wlref_n_bonds.restype = ctypes.c_int
        L.wlref_n_bins.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.wlref_n_bins.restype = ctypes.c_int
        L.wlref_histogram_flat.argtypes = [P(ctypes.c_uint64), P(ctypes.c_uint8), ctypes.c_int,
                                           ctypes.c_double, ctypes.c_int, P(ctypes.c_int)]
        L.wlref_histogram_flat.restype = ctypes.c_int
        L.wlref_walker_create.argtypes = [P(WlrefParams), P(ctypes.c_void_p)]
        L.wlref_walker_create.restype = ctypes.c_int
        L.wlref_walker_destroy.argtypes = [ctypes.c_void_p]
        L.wlref_walker_destroy.restype = None
        L.wlref_walker_set_debug.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.wlref_walker_set_debug.restype = None
        L.wlref_walker_advance.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.wlref_walker_advance.restype = ctypes.c_int
        L.wlref_walker_info.argtypes = [ctypes.c_void_p, P(WlrefInfo)]
        L.wlref_walker_info.restype = ctypes.c_int
        L.wlref_walker_copy.argtypes = [ctypes.c_void_p, P(ctypes.c_double), P(ctypes.c_uint64),
                                        P(ctypes.c_uint8), P(ctypes.c_uint8), P(ctypes.c_int32),
                                        P(ctypes.c_int32)]
        L.wlref_walker_copy.restype = ctypes.c_int
        L.wlref_line_run.argtypes = [P(WlrefParams), P(ctypes.c_double), ctypes.c_size_t, P(WlrefInfo)]
        L.wlref_line_run.restype = ctypes.c_int
        L.wlref_assemble.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     P(ctypes.c_double),
                                     P(ctypes.c_size_t), P(ctypes.c_double), P(ctypes.c_double)]
        L.wlref_assemble.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().wlref_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def exp_fixed(x: float) -> float:
    return lib().wlref_exp_fixed(float(x))


SQUARE, TRIANGULAR, HONEYCOMB = 0, 1, 2


def count_k(L: int, spins, boundary: int = 0, lattice: int = SQUARE) -> int:
    s = np.ascontiguousarray(spins, dtype=np.uint8)
    if boundary or lattice:
        return lib().wlref_count_k_geo(L, lattice, boundary, _ptr(s, ctypes.c_uint8))
    return lib().wlref_count_k(L, _ptr(s, ctypes.c_uint8))


def n_bonds(L: int, boundary: int = 0, lattice: int = SQUARE) -> int:
    """N_B of the oracle's lattice (2N periodic square, 2L(L-1) open square, ...)."""
    return lib().wlref_n_bonds(L, lattice, boundary)


def n_bins(L: int, ell: int, boundary: int = 0, lattice: int = SQUARE) -> int:
    """Bins of line ell (bin q <-> k = 2q on periodic square and triangular
    lattices, k = q otherwise)."""
    return lib().wlref_n_bins(L, lattice, boundary, ell)


HELD = 2   # boundary: periodic, the last row held up


def free_sites(L: int, boundary: int = 0) -> int:
    """Sites the walk moves: N, or N - L with the last row held up."""
    return L * L - (L if boundary == HELD else 0)


def bin_shift(boundary: int = 0, lattice: int = SQUARE) -> int:
    return 1 if (boundary != 1 and lattice in (SQUARE, TRIANGULAR)) else 0


def histogram_flat(h, vis, flatness, nprev):
    """(flat, n_visited) of the oracle's flatness test on a given histogram."""
    hh = np.ascontiguousarray(h, dtype=np.uint64)
    vv = np.ascontiguousarray(vis, dtype=np.uint8)
    n = ctypes.c_int(0)
    f = lib().wlref_histogram_flat(_ptr(hh, ctypes.c_uint64), _ptr(vv, ctypes.c_uint8), hh.size,
                                   float(flatness), int(nprev), ctypes.byref(n))
    return bool(f), n.value


def default_check_interval(L: int) -> int:
    return 16 * L * L


def make_params(L, ell, seed, walker=0, lnf0=1.0, lnf_min=1e-6, flatness=0.8, check_interval=0,
                reset_checks=0, boundary=0, lattice=SQUARE):
    return WlrefParams(L=L, ell=ell, seed=seed, walker=walker, reset_checks=reset_checks, lnf0=lnf0,
                       lnf_min=lnf_min, flatness=flatness, check_interval=check_interval, boundary=boundary,
                       lattice=lattice)


@dataclass
class WalkerState:
    attempts: int
    accepts: int
    stages: int
    done: bool
    k: int
    nb: int
    nprev: int
    lnf: float
    lng: np.ndarray
    h: np.ndarray
    vis: np.ndarray
    spins: np.ndarray
    up: np.ndarray
    dn: np.ndarray


class Walker:
    """One oracle walker; ``advance(n)`` runs up to n more proposals."""

    def __init__(self, L, ell, seed, walker=0, lnf0=1.0, lnf_min=1e-6, flatness=0.8,
                 check_interval=0, debug=False, reset_checks=0, boundary=0, lattice=SQUARE):
        self.L, self.ell, self.boundary = L, ell, boundary
        self.params = make_params(L, ell, seed, walker, lnf0, lnf_min, flatness, check_interval,
                                  reset_checks, boundary, lattice)
        h = ctypes.c_void_p()
        st = lib().wlref_walker_create(ctypes.byref(self.params), ctypes.byref(h))
        if st != 0:
            raise ValueError(f"wlref_walker_create: status {st}")
        self._h = h
        if debug:
            lib().wlref_walker_set_debug(self._h, 1)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().wlref_walker_destroy(h)
            self._h = None

    def advance(self, n: int = (1 << 64) - 1) -> bool:
        st = lib().wlref_walker_advance(self._h, n)
        if st < 0:
            raise RuntimeError(f"wlref_walker_advance: status {st}")
        return st == 1

    def info(self) -> WlrefInfo:
        inf = WlrefInfo()
        lib().wlref_walker_info(self._h, ctypes.byref(inf))
        return inf

    def state(self) -> WalkerState:
        inf = self.info()
        N = self.L * self.L
        lng = np.zeros(inf.nb, dtype=np.float64)
        h = np.zeros(inf.nb, dtype=np.uint64)
        vis = np.zeros(inf.nb, dtype=np.uint8)
        spins = np.zeros(N, dtype=np.uint8)
        Nf = free_sites(self.L, self.boundary)
        up = np.zeros(max(self.ell, 1), dtype=np.int32)
        dn = np.zeros(max(Nf - self.ell, 1), dtype=np.int32)
        lib().wlref_walker_copy(self._h, _ptr(lng, ctypes.c_double), _ptr(h, ctypes.c_uint64),
                                _ptr(vis, ctypes.c_uint8), _ptr(spins, ctypes.c_uint8),
                                _ptr(up, ctypes.c_int32), _ptr(dn, ctypes.c_int32))
        return WalkerState(inf.attempts, inf.accepts, inf.stages, bool(inf.done), inf.k, inf.nb,
                           inf.nprev, inf.lnf, lng, h, vis, spins, up[:self.ell], dn[:Nf - self.ell])


def line_run(L, ell, seed, walker=0, lnf0=1.0, lnf_min=1e-6, flatness=0.8, check_interval=0,
             reset_checks=0, boundary=0, lattice=SQUARE):
    """Run one walker to completion; returns (lng with -inf where unvisited, info)."""
    p = make_params(L, ell, seed, walker, lnf0, lnf_min, flatness, check_interval, reset_checks, boundary,
                    lattice)
    nb = n_bins(L, ell, boundary, lattice)
    out = np.zeros(nb, dtype=np.float64)
    inf = WlrefInfo()
    st = lib().wlref_line_run(ctypes.byref(p), _ptr(out, ctypes.c_double), nb, ctypes.byref(inf))
    if st != 0:
        raise ValueError(f"wlref_line_run: status {st}")
    return out, inf


def assemble(L: int, lines: list, n_lines: int | None = None, boundary: int = 0, lattice: int = SQUARE):
    """lines[i] is an array (W, nb(i)) (or (nb(i),) for W = 1) of per-walker
    ln g for ell = i.

    Returns (lng_kl, lng_k) with N+1 rows and (N_B >> s) + 1 columns,
    column q <-> k = q << s (s = bin_shift(boundary, lattice)): the periodic
    square lattice gives (N+1, N+1) with k = 2q, the open one N_B + 1 columns.
    """
    N = L * L
    n_lines = len(lines) if n_lines is None else n_lines
    W = 1 if np.asarray(lines[0]).ndim == 1 else np.asarray(lines[0]).shape[0]
    flat, offsets, off = [], [], 0
    for i in range(n_lines):
        a = np.asarray(lines[i], dtype=np.float64).reshape(W, -1)
        offsets.append(off)
        flat.append(a.reshape(-1))
        off += a.size
    buf = np.ascontiguousarray(np.concatenate(flat))
    offs = np.asarray(offsets, dtype=np.uintp)
    ncol = (n_bonds(L, boundary, lattice) >> bin_shift(boundary, lattice)) + 1
    kl = np.zeros((N + 1, ncol), dtype=np.float64)
    gk = np.zeros(ncol, dtype=np.float64)
    st = lib().wlref_assemble(L, lattice, boundary, n_lines, W, _ptr(buf, ctypes.c_double), _ptr(offs, ctypes.c_size_t),
                              _ptr(kl, ctypes.c_double), _ptr(gk, ctypes.c_double))
    if st != 0:
        raise ValueError(f"wlref_assemble: status {st}")
    return kl, gk


def log_binomial(n: int, r: int) -> float:
    return math.lgamma(n + 1) - math.lgamma(r + 1) - math.lgamma(n - r + 1)
