"""Exact degeneracies of the L x L periodic Ising lattice.

TEST INFRASTRUCTURE ONLY: exact references that pin the oracle and, through
it, the GPU library.  Nothing in the product imports this module.

Three independent routes to the degeneracies of Eq. 2:

* ``brute_force(L)`` -- every one of the 2^N configurations (L = 4).
* ``transfer_matrix(L)`` -- exact g(k, ell) by a site-by-site transfer
  matrix (``exact_tm.c``), L <= 8.  The paper names a transfer-matrix method
  as its source of exact surfaces in a field.
* ``kaufman_gk(L)`` -- exact zero-field g_k = sum over ell of g(k, ell), the
  quantity the paper compares its summed lines with (Beale's expansion of
  Kaufman's finite-torus partition function).  Built here from the
  Pfaffian form of the torus partition function (the high-temperature
  expansion as four Pfaffians with periodic/antiperiodic boundary
  conditions, whose factors are diagonal in Fourier space), rewritten in
  x = exp(-2K) so that it becomes the polynomial sum_k g_k x^k directly,
  evaluated exactly modulo many primes and recombined by the Chinese
  remainder theorem.

Plus ``closed_forms(L)``: degeneracies that follow by hand-counting for the
lowest lines and the spectrum ends named in the paper's discussion of the
ground and Neel states.
"""
from __future__ import annotations

import ctypes
import math
import os
from functools import lru_cache

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# Brute force
# ---------------------------------------------------------------------------
def bonds(L: int, boundary: int = 0, lattice: int = 0) -> list:
    """The bonds (i, j), i < j, of the L x L grid: lattice 0 square (each site
    bonded to the site on its right and the one below), 1 triangular (also
    the one below-right), 2 honeycomb in brick-wall form (right always; below
    only from sites with r + c even).  Periodic lattices wrap; open ones
    drop the bonds that would cross an edge; boundary 2 (the last row held
    up) has the periodic bonds."""
    out = set()
    for r in range(L):
        for c in range(L):
            i = r * L + c
            cand = [(r, c + 1)]
            if lattice != 2 or (r + c) % 2 == 0:
                cand.append((r + 1, c))
            if lattice == 1:
                cand.append((r + 1, c + 1))
            for rr, cc in cand:
                if boundary == 1 and (rr >= L or cc >= L):
                    continue
                j = (rr % L) * L + cc % L
                out.add((min(i, j), max(i, j)))
    return sorted(out)


def brute_force(L: int, boundary: int = 0, lattice: int = 0) -> np.ndarray:
    """g[ell, k] for the L x L lattice by enumerating all 2^N states (2^(N-L)
    with the last row held up, boundary 2).

    Each configuration is an integer whose bit i is the spin of site
    i = row*L + col (1 = up); k counts bonds whose two ends differ (Eq. 2).
    The bonds are those of ``bonds(L, boundary, lattice)``: periodic square
    has 2N of them, open square 2L(L-1).  Feasible for N <= 20 or so (L = 4:
    65536 states).
    """
    N = L * L
    if N > 24:
        raise ValueError("brute force only for N <= 24")
    # boundary 2: only the first N - L sites vary, the last row is up, and
    # ell counts the up spins among the free sites
    Nf = N - L if boundary == 2 else N
    states = np.arange(1 << Nf, dtype=np.int64)
    bits = ((states[:, None] >> np.arange(N, dtype=np.int64)[None, :]) & 1).astype(np.int8)
    bits[:, Nf:] = 1
    ell = bits[:, :Nf].sum(axis=1)
    k = np.zeros(1 << Nf, dtype=np.int64)
    bl = bonds(L, boundary, lattice)
    for i, j in bl:
        k += bits[:, i] != bits[:, j]
    g = np.zeros((N + 1, len(bl) + 1), dtype=np.int64)
    np.add.at(g, (ell, k), 1)
    return g


# ---------------------------------------------------------------------------
# Transfer matrix (C)
# ---------------------------------------------------------------------------
def _tm_lib():
    path = os.path.join(_HERE, "libexact_tm.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    lib.wlref_exact_tm.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
    lib.wlref_exact_tm.restype = ctypes.c_int
    return lib


@lru_cache(maxsize=None)
def _transfer_matrix_cached(L: int) -> bytes:
    N = L * L
    out = np.zeros((N + 1, 2 * N + 1), dtype=np.uint64)
    st = _tm_lib().wlref_exact_tm(L, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if st != 0:
        raise RuntimeError(f"wlref_exact_tm failed with {st}")
    return out.tobytes()


def transfer_matrix(L: int) -> np.ndarray:
    """Exact g[ell, k] (uint64) for L <= 8 by the transfer matrix."""
    N = L * L
    return np.frombuffer(_transfer_matrix_cached(L), dtype=np.uint64).reshape(N + 1, 2 * N + 1).copy()


# ---------------------------------------------------------------------------
# Zero-field exact g_k (Kaufman / Beale), modular evaluation + CRT
# ---------------------------------------------------------------------------
def _is_prime(n: int) -> bool:
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def _prime_factors(n: int):
    f, d = set(), 2
    while d * d <= n:
        while n % d == 0:
            f.add(d)
            n //= d
        d += 1
    if n > 1:
        f.add(n)
    return f


def _generator(p: int) -> int:
    fs = _prime_factors(p - 1)
    g = 2
    while any(pow(g, (p - 1) // q, p) == 1 for q in fs):
        g += 1
    return g


def _ntt_inverse(vals: np.ndarray, p: int, root: int) -> np.ndarray:
    """Coefficients c_j of the polynomial with P(root^i) = vals[i] (mod p).

    A plain O(S log S) iterative transform over Z/p with the inverse root;
    all products stay below 2^62.
    """
    S = vals.shape[0]
    a = vals.astype(np.int64).copy()
    # bit-reversal permutation
    bits = S.bit_length() - 1
    idx = np.arange(S)
    rev = np.zeros(S, dtype=np.int64)
    for b in range(bits):
        rev |= ((idx >> b) & 1) << (bits - 1 - b)
    a = a[rev]
    inv_root = pow(root, p - 2, p)
    length = 2
    while length <= S:
        w_len = pow(inv_root, S // length, p)
        half = length // 2
        w = np.ones(half, dtype=np.int64)
        for j in range(1, half):
            w[j] = w[j - 1] * w_len % p
        a = a.reshape(-1, length)
        u = a[:, :half].copy()
        v = a[:, half:] * w[None, :] % p
        a[:, :half] = (u + v) % p
        a[:, half:] = (u - v) % p
        a = a.reshape(-1)
        length *= 2
    inv_S = pow(S, p - 2, p)
    return a * inv_S % p


def _torus_poly_mod(L: int, p: int, S: int, root_S: int, zeta: int) -> np.ndarray:
    """sum_k g_k x^k evaluated at x = root_S^i, i < S, modulo p.

    Pfaffian form: sum_k g_k x^k = (Pf00 + Pf01 + Pf10 + Pf11) / 2 with, for
    boundary phases (a, b) in {0,1}^2, Pf_ab the product over one
    representative of each pair {(p, q), (-p-a, -q-b)} of
        phi(x; c) = (1 + x^2)^2 - x (1 - x^2) c,
        c = 2 cos(pi (2p + a) / L) + 2 cos(pi (2q + b) / L),
    and, for the four self-paired momenta of the periodic-periodic term, the
    square roots (1 - 2x - x^2) [c = 4], (1 + x^2) [c = 0, twice] and
    (1 + 2x - x^2) [c = -4].  2 cos(pi j / L) is zeta^j + zeta^-j with zeta
    a primitive 2L-th root of unity mod p.
    """
    xs = np.ones(S, dtype=np.int64)
    for i in range(1, S):
        xs[i] = xs[i - 1] * root_S % p
    x2 = xs * xs % p
    A = (1 + x2) % p
    A = A * A % p                       # (1 + x^2)^2
    B = xs * ((1 - x2) % p) % p         # x (1 - x^2)
    twocos = [(pow(zeta, j, p) + pow(zeta, (2 * L - j) % (2 * L), p)) % p for j in range(2 * L)]

    def pf(a: int, b: int) -> np.ndarray:
        # representatives: (p, q) with (p, q) < (-p-a mod L, -q-b mod L) lexicographically
        counts = {}
        self_paired = []
        for pp in range(L):
            for qq in range(L):
                mp, mq = (-pp - a) % L, (-qq - b) % L
                if (pp, qq) == (mp, mq):
                    self_paired.append((pp, qq))
                    continue
                if (pp, qq) > (mp, mq):
                    continue
                c = (twocos[(2 * pp + a) % (2 * L)] + twocos[(2 * qq + b) % (2 * L)]) % p
                counts[c] = counts.get(c, 0) + 1
        out = np.ones(S, dtype=np.int64)
        for c, mult in counts.items():
            f = (A - B * c % p) % p
            acc = np.ones(S, dtype=np.int64)
            base, e = f, mult
            while e:
                if e & 1:
                    acc = acc * base % p
                base = base * base % p
                e >>= 1
            out = out * acc % p
        for (pp, qq) in self_paired:
            cval = math.cos(math.pi * (2 * pp + a) / L) + math.cos(math.pi * (2 * qq + b) / L)
            if cval > 1.5:
                f = (1 - 2 * xs - x2) % p
            elif cval < -1.5:
                f = (1 + 2 * xs - x2) % p
            else:
                f = (1 + x2) % p
            out = out * f % p
        return out

    p00 = pf(0, 0)
    p01 = pf(0, 1)
    p10 = pf(1, 0)
    p11 = pf(1, 1)
    inv2 = pow(2, p - 2, p)
    return (p00 + p01 + p10 + p11) % p * inv2 % p


@lru_cache(maxsize=None)
def kaufman_gk(L: int) -> tuple:
    """Exact zero-field degeneracies g_k, k = 0..2N, as Python ints (even L)."""
    if L < 4 or L % 2:
        raise ValueError("even L >= 4")
    N = L * L
    deg = 2 * N
    S = 1
    while S <= deg:
        S *= 2
    modulus = S * (2 * L) // math.gcd(S, 2 * L)
    bound_bits = N + 4           # g_k <= 2^N
    primes = []
    prod = 1
    c = (1 << 31) // modulus
    while prod.bit_length() <= bound_bits + 1:
        cand = c * modulus + 1
        c -= 1
        if cand < (1 << 31) and _is_prime(cand):
            primes.append(cand)
            prod *= cand
    residues = []
    for p in primes:
        g = _generator(p)
        root_S = pow(g, (p - 1) // S, p)
        zeta = pow(g, (p - 1) // (2 * L), p)
        vals = _torus_poly_mod(L, p, S, root_S, zeta)
        coef = _ntt_inverse(vals, p, root_S)
        residues.append(coef)
    # Chinese remainder reconstruction, coefficient by coefficient
    result = []
    for kk in range(deg + 1):
        x = 0
        m = 1
        for p, res in zip(primes, residues):
            r = int(res[kk])
            # x' = x + m * t with x' = r (mod p)
            t = ((r - x) * pow(m % p, p - 2, p)) % p
            x += m * t
            m *= p
        result.append(x)
    for kk in range(deg + 1, S):
        for res in residues:
            if int(res[kk]) != 0:
                raise ArithmeticError("coefficient beyond degree 2N is not zero")
    return tuple(result)


def log_kaufman_gk(L: int) -> np.ndarray:
    """ln g_k for k = 0..2N (-inf where g_k = 0)."""
    g = kaufman_gk(L)
    return np.array([math.log(v) if v > 0 else -math.inf for v in g])


# ---------------------------------------------------------------------------
# Closed forms
# ---------------------------------------------------------------------------
def closed_forms(L: int) -> dict:
    """Degeneracies that follow by direct counting, {(k, ell): g}.

    ell = 0: the all-down state, k = 0.
    ell = 1: one up spin, four broken bonds: g(4, 1) = N.
    ell = 2: the two up spins adjacent (2N pairs) break 6 bonds, otherwise 8.
    ell = 3: three in a straight or bent chain (2N straight, 4N bent: each
      chain counted by its middle site) break 8; exactly one adjacent pair
      (an adjacent pair, 2N of them, plus a third spin touching neither, i.e.
      not among the N - 2 - 6 sites that are either of the pair or one of
      their 6 other neighbours) breaks 10; no adjacency breaks 12.
    ell = N/2: the two Neel states break every bond (k = 2N); the ground
      state of the line is a straight band of L/2 full rows (or columns) of up
      spins, L positions times 2 orientations, with two flat interfaces of L
      broken bonds each (k = 2L).
    """
    N = L * L
    out = {}
    out[(0, 0)] = 1
    out[(4, 1)] = N
    out[(6, 2)] = 2 * N
    out[(8, 2)] = math.comb(N, 2) - 2 * N
    out[(8, 3)] = 6 * N
    out[(10, 3)] = 2 * N * (N - 8)
    out[(12, 3)] = math.comb(N, 3) - 6 * N - 2 * N * (N - 8)
    out[(2 * N, N // 2)] = 2
    out[(2 * L, N // 2)] = 2 * L
    return out
