"""Python binding of libwl (include/wl.h): argument marshalling only.

Every step of the walk and of the assembly runs in the HIP kernels behind
the C ABI; PyTorch supplies device memory (workspace and output tensors) and
streams.  The binding refuses to run without the compiled library.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libwl.so")

WL_OK, WL_EINVAL, WL_ENOMEM, WL_EDEVICE, WL_EBUSY, WL_ECANCELED = 0, -1, -2, -3, -4, -5


class WlError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class LineParamsC(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("ell", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("walker", ctypes.c_uint32), ("reset_checks", ctypes.c_uint32),
                ("lnf0", ctypes.c_double), ("lnf_min", ctypes.c_double),
                ("flatness", ctypes.c_double), ("check_interval", ctypes.c_uint64),
                ("boundary", ctypes.c_uint32), ("lattice", ctypes.c_uint32)]


class LineStatsC(ctypes.Structure):
    _fields_ = [("attempts", ctypes.c_uint64), ("accepts", ctypes.c_uint64),
                ("stages", ctypes.c_uint32), ("done", ctypes.c_uint32),
                ("k", ctypes.c_int32), ("nb", ctypes.c_int32), ("final_lnf", ctypes.c_double)]


class TuningC(ctypes.Structure):
    _fields_ = [("walkers_per_wave", ctypes.c_int32), ("placement", ctypes.c_int32),
                ("round_kproposals", ctypes.c_int32), ("tail_walkers", ctypes.c_int32),
                ("wide_placement", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class JobStatsC(ctypes.Structure):
    _fields_ = [("submit_s", ctypes.c_double), ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("attempts", ctypes.c_uint64), ("lines", ctypes.c_uint32), ("walkers", ctypes.c_uint32),
                ("status", ctypes.c_int32), ("reserved", ctypes.c_uint32)]


STATS_DTYPE = np.dtype([("attempts", "<u8"), ("accepts", "<u8"), ("stages", "<u4"), ("done", "<u4"),
                        ("k", "<i4"), ("nb", "<i4"), ("final_lnf", "<f8")])

# The exported symbols, as declared in include/wl.h.
EXPORTS = ("wl_line_run", "wl_line_run_ex", "wl_batch_workspace_size", "wl_batch_create",
           "wl_batch_advance", "wl_batch_run", "wl_batch_run_to_end", "wl_batch_stats", "wl_batch_lng_offsets",
           "wl_batch_lng", "wl_batch_read_walker", "wl_batch_destroy", "wl_batch_run_async", "wl_assemble",
           "wl_assemble_ex",
           "wl_server_create", "wl_server_submit", "wl_server_poll", "wl_server_wait",
           "wl_server_job_stats", "wl_server_fetch", "wl_server_destroy",
           "wl_thermo", "wl_thermo_ex", "wl_thermo_noalloc", "wl_selfcheck_accept", "wl_selfcheck_threshold", "wl_selfcheck_exp",
           "wl_strerror", "wl_last_error")

_lib = None


def lib():
    """Load libwl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, c = ctypes.POINTER, ctypes
    L.wl_strerror.argtypes, L.wl_strerror.restype = [c.c_int], c.c_char_p
    L.wl_last_error.argtypes, L.wl_last_error.restype = [], c.c_char_p
    L.wl_line_run.argtypes = [c.c_int, c.c_int, c.c_uint64, c.c_double, c.c_double, c.c_double,
                              P(c.c_double), c.c_size_t, P(LineStatsC)]
    L.wl_line_run_ex.argtypes = [P(LineParamsC), P(c.c_double), c.c_size_t, P(LineStatsC)]
    L.wl_batch_workspace_size.argtypes = [P(LineParamsC), c.c_size_t, P(c.c_size_t)]
    L.wl_batch_create.argtypes = [P(LineParamsC), c.c_size_t, P(TuningC), c.c_void_p, c.c_size_t,
                                  c.c_void_p, P(c.c_void_p)]
    L.wl_batch_advance.argtypes = [c.c_void_p, c.c_uint64, c.c_void_p]
    L.wl_batch_run_to_end.argtypes = [c.c_void_p, c.c_uint64, c.c_void_p]
    L.wl_batch_run.argtypes = [c.c_void_p, c.c_uint64, c.c_uint32, P(c.c_uint32), c.c_void_p]
    L.wl_batch_stats.argtypes = [c.c_void_p, c.c_void_p, c.c_void_p]
    L.wl_batch_lng_offsets.argtypes = [c.c_void_p, P(c.c_size_t)]
    L.wl_batch_lng.argtypes = [c.c_void_p, c.c_void_p, c.c_void_p]
    L.wl_batch_read_walker.argtypes = [c.c_void_p, c.c_size_t, P(c.c_uint8), P(c.c_uint16), P(c.c_uint16),
                                       P(c.c_double), P(c.c_uint64), P(LineStatsC), P(c.c_int32)]
    L.wl_batch_destroy.argtypes = [c.c_void_p]
    L.wl_batch_run_async.argtypes = [P(LineParamsC), c.c_size_t, P(TuningC), c.c_void_p, c.c_size_t, c.c_void_p,
                                     c.c_void_p, c.c_void_p]
    L.wl_assemble.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_void_p, c.c_void_p, c.c_void_p,
                              c.c_void_p, c.c_void_p]
    L.wl_assemble_ex.argtypes = [c.c_int, c.c_int, c.c_int, c.c_int, c.c_int, c.c_void_p, c.c_void_p,
                                 c.c_void_p, c.c_void_p, c.c_void_p]
    L.wl_server_create.argtypes = [c.c_size_t, P(TuningC), P(c.c_void_p)]
    L.wl_server_submit.argtypes = [c.c_void_p, c.c_int, c.c_int, c.c_uint64, c.c_double, c.c_double, c.c_double,
                                   P(c.c_uint64)]
    L.wl_server_poll.argtypes = [c.c_void_p, c.c_uint64, P(c.c_int)]
    L.wl_server_wait.argtypes = [c.c_void_p, c.c_uint64, c.c_double]
    L.wl_server_job_stats.argtypes = [c.c_void_p, c.c_uint64, P(JobStatsC)]
    L.wl_server_fetch.argtypes = [c.c_void_p, c.c_uint64, P(c.c_double), c.c_size_t]
    L.wl_server_destroy.argtypes = [c.c_void_p]
    L.wl_selfcheck_accept.argtypes = [c.c_double, c.c_double, c.c_uint64, P(c.c_double)]
    L.wl_thermo.argtypes = [c.c_int, c.c_int, c.c_void_p, c.c_double, c.c_size_t, c.c_void_p, c.c_void_p,
                            c.c_void_p, c.c_void_p, c.c_void_p]
    L.wl_thermo_ex.argtypes = [c.c_int, c.c_int, c.c_int, c.c_void_p, c.c_double, c.c_size_t, c.c_void_p,
                               c.c_void_p, c.c_void_p, c.c_void_p, c.c_void_p]
    L.wl_selfcheck_threshold.argtypes = [c.c_double, c.c_double, c.c_uint64, P(c.c_uint64), P(c.c_uint64)]
    L.wl_thermo_noalloc.argtypes = [c.c_int, c.c_int, c.c_int, c.c_void_p, c.c_double, c.c_size_t, c.c_void_p,
                                    c.c_void_p, c.c_void_p, c.c_void_p, c.c_void_p]
    L.wl_selfcheck_exp.argtypes = [c.c_void_p, c.c_void_p, c.c_size_t, c.c_void_p]
    for name in EXPORTS:
        if name not in ("wl_strerror", "wl_last_error"):
            getattr(L, name).restype = c.c_int
    _lib = L
    return L


def _check(status: int, where: str) -> None:
    if status != WL_OK:
        raise WlError(status, where, lib().wl_last_error().decode())


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


@dataclass
class LineParams:
    L: int
    ell: int
    seed: int = 1
    walker: int = 0
    lnf0: float = 1.0
    lnf_min: float = 1e-8
    flatness: float = 0.8
    check_interval: int = 0
    reset_checks: int = 0
    boundary: int = 0
    lattice: int = 0

    def to_c(self) -> LineParamsC:
        return to_c(self)

    @property
    def nb(self) -> int:
        return n_bins(self.L, self.ell, self.boundary, self.lattice)


SQUARE, TRIANGULAR, HONEYCOMB = 0, 1, 2
PERIODIC, OPEN, HELD = 0, 1, 2      # boundary; HELD: periodic, the last row held up
_DEGREE = {SQUARE: 4, TRIANGULAR: 6, HONEYCOMB: 3}


def n_bonds(L: int, boundary: int = 0, lattice: int = SQUARE) -> int:
    """N_B (include/wl.h, Conventions); the held row keeps the periodic bonds."""
    N, o = L * L, L * (L - 1)
    op = boundary == OPEN
    if lattice == TRIANGULAR:
        return 2 * o + (L - 1) ** 2 if op else 3 * N
    if lattice == HONEYCOMB:
        return o + o // 2 if op else 3 * N // 2
    return 2 * o if op else 2 * N


def bin_shift(boundary: int = 0, lattice: int = SQUARE) -> int:
    """Bin q holds k = q << shift: 1 on periodic lattices of even degree."""
    return 1 if boundary != OPEN and _DEGREE[lattice] % 2 == 0 else 0


def free_sites(L: int, boundary: int = 0) -> int:
    """Sites the walk moves: N, or N - L with the last row held up."""
    return L * L - (L if boundary == HELD else 0)


def n_bins(L: int, ell: int, boundary: int = 0, lattice: int = SQUARE) -> int:
    """Bins of a line (include/wl.h, Conventions): (min(z m, N_B) >> shift) + 1,
    m = the smaller of the up and down spin counts; 2m + 1 on the periodic
    square lattice."""
    nup = ell + (L if boundary == HELD else 0)
    m = min(nup, L * L - nup)
    return (min(_DEGREE[lattice] * m, n_bonds(L, boundary, lattice)) >> bin_shift(boundary, lattice)) + 1


def n_columns(L: int, boundary: int = 0, lattice: int = SQUARE) -> int:
    """Columns of an assembled plane: (N_B >> shift) + 1 (N + 1 periodic square)."""
    return (n_bonds(L, boundary, lattice) >> bin_shift(boundary, lattice)) + 1


def to_c(p) -> LineParamsC:
    """wl_line_params from any object with the fields of LineParams."""
    return LineParamsC(L=p.L, ell=p.ell, seed=p.seed, walker=p.walker,
                       reset_checks=getattr(p, "reset_checks", 0), lnf0=p.lnf0, lnf_min=p.lnf_min,
                       flatness=p.flatness, check_interval=p.check_interval,
                       boundary=getattr(p, "boundary", 0), lattice=getattr(p, "lattice", 0))


def _nb(p) -> int:
    return n_bins(p.L, p.ell, getattr(p, "boundary", 0), getattr(p, "lattice", 0))


def _stream_handle(stream) -> ctypes.c_void_p:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def line_run(L: int, ell: int, seed: int, lnf0: float = 1.0, lnf_min: float = 1e-6, flatness: float = 0.8):
    """wl_line_run: one walker to completion, host output. Returns (ln g, stats dict)."""
    N = L * L
    nb = 2 * min(ell, N - ell) + 1 if 0 <= ell <= N else 1
    out = np.zeros(max(nb, 1), dtype=np.float64)
    st = LineStatsC()
    _check(lib().wl_line_run(L, ell, seed, lnf0, lnf_min, flatness, _ptr(out, ctypes.c_double), out.size,
                             ctypes.byref(st)), "wl_line_run")
    return out, {f: getattr(st, f) for f, _ in LineStatsC._fields_}


def line_run_ex(p):
    out = np.zeros(_nb(p), dtype=np.float64)
    st = LineStatsC()
    cp = to_c(p)
    _check(lib().wl_line_run_ex(ctypes.byref(cp), _ptr(out, ctypes.c_double), out.size, ctypes.byref(st)),
           "wl_line_run_ex")
    return out, {f: getattr(st, f) for f, _ in LineStatsC._fields_}


@dataclass
class WalkerSnapshot:
    spins: np.ndarray
    up: np.ndarray
    dn: np.ndarray
    lng: np.ndarray
    h: np.ndarray
    stats: dict
    nprev: int


class Batch:
    """A set of independent walkers sharing one device workspace (wl_batch_*)."""

    def __init__(self, lines: list, walkers_per_wave: int = 0, placement: int = 0, stream=None,
                 device: str = "cuda", tail_walkers: int = 0, wide_placement: int = 0):
        import torch
        self.lines = list(lines)
        self._arr = (LineParamsC * len(self.lines))(*[to_c(p) for p in self.lines])
        nbytes = ctypes.c_size_t(0)
        _check(lib().wl_batch_workspace_size(self._arr, len(self.lines), ctypes.byref(nbytes)),
               "wl_batch_workspace_size")
        self.ws_bytes = nbytes.value
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self._tuning = TuningC(walkers_per_wave=walkers_per_wave, placement=placement, tail_walkers=tail_walkers,
                               wide_placement=wide_placement)
        h = ctypes.c_void_p()
        self.stream = stream
        _check(lib().wl_batch_create(self._arr, len(self.lines), ctypes.byref(self._tuning),
                                     ctypes.c_void_p(self.workspace.data_ptr()), self.ws_bytes,
                                     _stream_handle(stream), ctypes.byref(h)), "wl_batch_create")
        self._h = h
        offs = np.zeros(len(self.lines) + 1, dtype=np.uintp)
        _check(lib().wl_batch_lng_offsets(self._h, _ptr(offs, ctypes.c_size_t)), "wl_batch_lng_offsets")
        self.lng_offsets = offs.astype(np.int64)

    def __len__(self):
        return len(self.lines)

    def advance(self, max_attempts: int) -> None:
        _check(lib().wl_batch_advance(self._h, max_attempts, _stream_handle(self.stream)), "wl_batch_advance")

    def run_to_end(self, chunk: int = 1 << 20) -> None:
        _check(lib().wl_batch_run_to_end(self._h, chunk, _stream_handle(self.stream)), "wl_batch_run_to_end")

    def run(self, chunk: int, max_chunks: int = 1) -> int:
        """wl_batch_run: up to max_chunks chunks; returns the walkers still walking."""
        active = ctypes.c_uint32(0)
        _check(lib().wl_batch_run(self._h, chunk, max_chunks, ctypes.byref(active), _stream_handle(self.stream)),
               "wl_batch_run")
        return active.value

    def stats(self) -> np.ndarray:
        import torch
        dev = torch.empty(len(self.lines) * STATS_DTYPE.itemsize, dtype=torch.uint8, device=self.workspace.device)
        _check(lib().wl_batch_stats(self._h, ctypes.c_void_p(dev.data_ptr()), _stream_handle(self.stream)),
               "wl_batch_stats")
        return np.frombuffer(dev.cpu().numpy().tobytes(), dtype=STATS_DTYPE)

    def lng(self):
        """Packed ln g of every walker (device tensor) and its offsets (numpy)."""
        import torch
        out = torch.empty(int(self.lng_offsets[-1]), dtype=torch.float64, device=self.workspace.device)
        _check(lib().wl_batch_lng(self._h, ctypes.c_void_p(out.data_ptr()), _stream_handle(self.stream)),
               "wl_batch_lng")
        return out, self.lng_offsets

    def lng_list(self) -> list:
        out, offs = self.lng()
        host = out.cpu().numpy()
        return [host[offs[i]:offs[i + 1]] for i in range(len(self.lines))]

    def read_walker(self, i: int) -> WalkerSnapshot:
        p = self.lines[i]
        N = p.L * p.L
        Nf = free_sites(p.L, getattr(p, "boundary", 0))
        spins = np.zeros(N, dtype=np.uint8)
        up = np.zeros(max(p.ell, 1), dtype=np.uint16)
        dn = np.zeros(max(Nf - p.ell, 1), dtype=np.uint16)
        lng = np.zeros(_nb(p), dtype=np.float64)
        h = np.zeros(_nb(p), dtype=np.uint64)
        st = LineStatsC()
        nprev = ctypes.c_int32(0)
        _check(lib().wl_batch_read_walker(self._h, i, _ptr(spins, ctypes.c_uint8), _ptr(up, ctypes.c_uint16),
                                          _ptr(dn, ctypes.c_uint16), _ptr(lng, ctypes.c_double),
                                          _ptr(h, ctypes.c_uint64), ctypes.byref(st), ctypes.byref(nprev)),
               "wl_batch_read_walker")
        return WalkerSnapshot(spins, up[:p.ell], dn[:Nf - p.ell], lng, h,
                              {f: getattr(st, f) for f, _ in LineStatsC._fields_}, nprev.value)

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().wl_batch_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_async(lines: list, stream=None, placement: int = 0, walkers_per_wave: int = 0, device: str = "cuda"):
    """wl_batch_run_async: every walker of `lines` to the end, enqueued on the
    stream.  Returns (packed ln g tensor, offsets (numpy, n + 1), stats
    tensor of raw wl_line_stats bytes, workspace tensor); the tensors are
    valid once the stream has passed the call's work."""
    import torch
    arr = (LineParamsC * len(lines))(*[to_c(p) for p in lines])
    nbytes = ctypes.c_size_t(0)
    _check(lib().wl_batch_workspace_size(arr, len(lines), ctypes.byref(nbytes)), "wl_batch_workspace_size")
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
    offs = np.zeros(len(lines) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([_nb(p) for p in lines])
    lng = torch.empty(int(offs[-1]), dtype=torch.float64, device=device)
    stats = torch.empty(len(lines) * STATS_DTYPE.itemsize, dtype=torch.uint8, device=device)
    tun = TuningC(walkers_per_wave=walkers_per_wave, placement=placement)
    _check(lib().wl_batch_run_async(arr, len(lines), ctypes.byref(tun), ctypes.c_void_p(ws.data_ptr()), nbytes.value,
                                    ctypes.c_void_p(lng.data_ptr()), ctypes.c_void_p(stats.data_ptr()),
                                    _stream_handle(stream)), "wl_batch_run_async")
    return lng, offs, stats, ws


def assemble(L: int, lng_lines, n_lines: int, W: int, offsets=None, stream=None, boundary: int = 0,
             lattice: int = SQUARE):
    """wl_assemble_ex on device tensors: returns (ln g(k, ell) [(N+1) x n_columns],
    ln g_k [n_columns])."""
    import torch
    if lng_lines.dtype != torch.float64 or not lng_lines.is_contiguous() or not lng_lines.is_cuda:
        raise ValueError("lng_lines must be a contiguous float64 device tensor")
    if offsets is not None and (offsets.dtype != torch.int64 or not offsets.is_contiguous()
                                or offsets.device != lng_lines.device or offsets.numel() < n_lines):
        raise ValueError("offsets must be a contiguous int64 tensor of n_lines entries on lng_lines' device")
    N = L * L
    dev = lng_lines.device
    ncol = n_columns(L, boundary, lattice)
    kl = torch.empty((N + 1, ncol), dtype=torch.float64, device=dev)
    gk = torch.empty(ncol, dtype=torch.float64, device=dev)
    offs = ctypes.c_void_p(offsets.data_ptr()) if offsets is not None else ctypes.c_void_p(0)
    _check(lib().wl_assemble_ex(L, lattice, boundary, n_lines, W, ctypes.c_void_p(lng_lines.data_ptr()), offs,
                                ctypes.c_void_p(kl.data_ptr()), ctypes.c_void_p(gk.data_ptr()),
                                _stream_handle(stream)), "wl_assemble_ex")
    return kl, gk


THERMO_FIELDS = ("lnZ", "e", "c", "m", "m_abs", "chi")


def thermo(L: int, lng_kl, beta, H, J: float = 1.0, stream=None, boundary: int = 0, lattice: int = SQUARE):
    """wl_thermo on a device tensor ln g(k, ell) [(N+1) x n_columns] at the points
    (beta[i], H[i]): returns (n x 6 float64 tensor on the device, columns
    THERMO_FIELDS; centre entropy S_C as a 1-element device tensor)."""
    import torch
    dev = lng_kl.device
    if lng_kl.dtype != torch.float64 or not lng_kl.is_contiguous():
        raise ValueError("lng_kl must be a contiguous float64 tensor")
    b = torch.as_tensor(beta, dtype=torch.float64).reshape(-1).to(dev).contiguous()
    h = torch.as_tensor(H, dtype=torch.float64).reshape(-1).to(dev).contiguous()
    if b.numel() != h.numel():
        raise ValueError("beta and H must have the same length")
    out = torch.empty((b.numel(), 6), dtype=torch.float64, device=dev)
    sc = torch.empty(1, dtype=torch.float64, device=dev)
    _check(lib().wl_thermo_ex(L, lattice, boundary, ctypes.c_void_p(lng_kl.data_ptr()), float(J), b.numel(),
                              ctypes.c_void_p(b.data_ptr()),
                              ctypes.c_void_p(h.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                              ctypes.c_void_p(sc.data_ptr()), _stream_handle(stream)), "wl_thermo_ex")
    return out, sc


def selfcheck_accept(d_lo: float = -80.0, d_hi: float = 0.0, n: int = 1 << 24) -> float:
    """wl_selfcheck_accept: largest relative error of the single-precision
    acceptance estimate over n points of [d_lo, d_hi] on the current device."""
    out = ctypes.c_double(0.0)
    _check(lib().wl_selfcheck_accept(d_lo, d_hi, n, ctypes.byref(out)), "wl_selfcheck_accept")
    return out.value


def selfcheck_threshold(d_lo: float = -800.0, d_hi: float = -1e-12, n: int = 1 << 18):
    """wl_selfcheck_threshold: (settled, wrong) decisions of the ln u bounds
    against the plain acceptance test on the current device."""
    settled, wrong = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(lib().wl_selfcheck_threshold(d_lo, d_hi, n, ctypes.byref(settled), ctypes.byref(wrong)),
           "wl_selfcheck_threshold")
    return settled.value, wrong.value


def exp_fixed_device(x, stream=None):
    """wl_selfcheck_exp: the device's exp_fixed at every element of x (a
    float64 tensor, copied to the device if needed); returns a device tensor."""
    import torch
    xd = torch.as_tensor(x, dtype=torch.float64).reshape(-1).cuda().contiguous()
    y = torch.empty_like(xd)
    _check(lib().wl_selfcheck_exp(ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(y.data_ptr()), xd.numel(),
                                  _stream_handle(stream)), "wl_selfcheck_exp")
    return y


class Server:
    """wl_server_*: DOS jobs (all lines of one L) served with continuous batching."""

    def __init__(self, hbm_budget_bytes: int, placement: int = 0, round_kproposals: int = 0,
                 walkers_per_wave: int = 0, tail_walkers: int = 0):
        self._tuning = TuningC(walkers_per_wave=walkers_per_wave, placement=placement,
                               round_kproposals=round_kproposals, tail_walkers=tail_walkers)
        h = ctypes.c_void_p()
        _check(lib().wl_server_create(hbm_budget_bytes, ctypes.byref(self._tuning), ctypes.byref(h)),
               "wl_server_create")
        self._h = h
        self.L_of = {}

    def submit(self, L: int, W: int = 1, seed: int = 1, lnf0: float = 1.0, lnf_min: float = 1e-7,
               flatness: float = 0.8) -> int:
        jid = ctypes.c_uint64(0)
        _check(lib().wl_server_submit(self._h, L, W, seed, lnf0, lnf_min, flatness, ctypes.byref(jid)),
               "wl_server_submit")
        self.L_of[jid.value] = L
        return jid.value

    def poll(self, job_id: int) -> bool:
        d = ctypes.c_int(0)
        _check(lib().wl_server_poll(self._h, job_id, ctypes.byref(d)), "wl_server_poll")
        return d.value == 1

    def wait(self, job_id: int, timeout_s: float = 600.0) -> None:
        _check(lib().wl_server_wait(self._h, job_id, timeout_s), "wl_server_wait")

    def job_stats(self, job_id: int) -> dict:
        st = JobStatsC()
        _check(lib().wl_server_job_stats(self._h, job_id, ctypes.byref(st)), "wl_server_job_stats")
        return {f: getattr(st, f) for f, _ in JobStatsC._fields_ if f != "reserved"}

    def fetch(self, job_id: int) -> np.ndarray:
        """wl_server_fetch: the job's assembled ln g(k, ell); the job's size is
        forgotten only once the fetch has succeeded, so a failed fetch can be
        repeated."""
        if job_id not in self.L_of:
            raise KeyError(f"job {job_id} was not submitted to this server or was already fetched")
        N = self.L_of[job_id] ** 2
        out = np.zeros((N + 1, N + 1), dtype=np.float64)
        _check(lib().wl_server_fetch(self._h, job_id, _ptr(out, ctypes.c_double), out.size), "wl_server_fetch")
        del self.L_of[job_id]
        return out

    def close(self) -> None:
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().wl_server_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
