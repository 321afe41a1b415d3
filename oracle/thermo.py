"""Thermodynamics from the assembled ln g(k, ell) (Eq. 2), plain numpy.

TEST INFRASTRUCTURE ONLY: the reference the GPU post-processing is checked
against.  Nothing in the product imports this module.

Eq. 2 writes the partition function of the Ising model in a field as
Z = sum over k, ell of g(k, ell) exp(-beta E(k, ell)), k the number of
antiparallel (unhappy) bonds.  With ell the number of up spins (the reading
the walk uses), the energy of such a state under the Hamiltonian of Eq. 1 is
E(k, ell) = -J (N_B - 2k) - H M with M = 2 ell - N; the field term printed in
Eq. 2, -H (N - 2 ell), is this with ell counting down spins instead (the
paper uses both meanings of ell; g(k, ell) = g(k, N - ell), so only the sign
of the field response depends on it).  On the L x L square lattice N_B = 2N
with periodic boundaries (k even, stored as q = k/2) and 2L(L-1) with open
ones (every k stored).
Everything below is a weighted average over the (k, ell) plane with weights
g(k, ell) exp(-beta E), written out directly (log-sum-exp for the scale).

The centre entropy of the paper's finite-size discussion (Eq. 5) is the
scaled DOS value at k = N_B / 2, ell = N / 2: S_C = ln g / N.
"""
from __future__ import annotations

import numpy as np

FIELDS = ("lnZ", "e", "c", "m", "m_abs", "chi")


def energy_magnetisation(L: int, boundary: int = 0, lattice: int = 0):
    """E(k, ell) for J = 1, H = 0 parts separately, on the assembled grid:
    returns (bond_term, field_term, M) as arrays indexed [ell, column]
    (column q <-> k = 2q periodic, column k open), so that
    E = J * bond_term + H * field_term."""
    from oracle import exact
    N = L * L
    NB = len(exact.bonds(L, boundary, lattice))
    s = 1 if (not boundary and lattice in (0, 1)) else 0    # column q <-> k = q << s
    ell = np.arange(N + 1, dtype=np.float64)[:, None]
    k = float(1 << s) * np.arange((NB >> s) + 1, dtype=np.float64)[None, :]
    bond = -(NB - 2.0 * k) + 0.0 * ell
    M = (2.0 * ell - N) + 0.0 * k
    field = -M
    return bond, field, M


def thermo(L: int, lng_kl: np.ndarray, beta: float, H: float, J: float = 1.0, boundary: int = 0,
           lattice: int = 0) -> dict:
    """ln Z and per-spin moments at (beta, H, J) from ln g[ell, q] (k = 2q,
    -inf where g = 0):
      lnZ;  e = <E>/N;  c = beta^2 var(E)/N;  m = <M>/N;  m_abs = <|M|>/N;
      chi = beta var(M)/N."""
    N = L * L
    bond, field, M = energy_magnetisation(L, boundary, lattice)
    lng = np.asarray(lng_kl, dtype=np.float64).reshape(bond.shape)
    E = J * bond + H * field
    ok = np.isfinite(lng)
    x = np.where(ok, lng - beta * E, -np.inf)
    mx = x[ok].max()
    w = np.where(ok, np.exp(x - mx), 0.0)
    Z0 = w.sum()
    Ebar = (w * E).sum() / Z0
    E2 = (w * E * E).sum() / Z0
    Mbar = (w * M).sum() / Z0
    M2 = (w * M * M).sum() / Z0
    Mabs = (w * np.abs(M)).sum() / Z0
    return {"lnZ": mx + np.log(Z0), "e": Ebar / N, "c": beta * beta * (E2 - Ebar * Ebar) / N,
            "m": Mbar / N, "m_abs": Mabs / N, "chi": beta * (M2 - Mbar * Mbar) / N}


def center_entropy(L: int, lng_kl: np.ndarray, boundary: int = 0, lattice: int = 0) -> float:
    """S_C = ln g(k = N_B/2, ell = N/2) / N (Eq. 5's quantity); the column of
    k = N_B/2 (rounded down to a column of the plane)."""
    bond, _, _ = energy_magnetisation(L, boundary, lattice)
    N = L * L
    lng = np.asarray(lng_kl, dtype=np.float64).reshape(bond.shape)
    return float(lng[N // 2, (bond.shape[1] - 1) // 2] / N)


def lng_from_counts(g_ell_k: np.ndarray, boundary: int = 0, lattice: int = 0) -> np.ndarray:
    """ln g on the assembled grid from integer counts g[ell, k] (k = 0..N_B),
    as the exact references return them: periodic square and triangular
    lattices keep the even k (odd k never occur) as q = k/2, the others keep
    every k."""
    if boundary or lattice == 2:
        g = g_ell_k.astype(np.float64)
    else:
        if np.any(g_ell_k[:, 1::2]):
            raise ValueError("odd k present")
        g = g_ell_k[:, 0::2].astype(np.float64)
    with np.errstate(divide="ignore"):
        return np.where(g > 0, np.log(np.where(g > 0, g, 1.0)), -np.inf)


def spin_enumeration(L: int, beta: float, H: float, J: float = 1.0, boundary: int = 0, lattice: int = 0) -> dict:
    """The same quantities by summing exp(-beta E) over all 2^N spin
    configurations with E from the spin Hamiltonian (Eq. 1):
    E = -J sum_<ij> S_i S_j - H sum_i S_i.  L = 4 only."""
    N = L * L
    if N > 20:
        raise ValueError("spin enumeration only for N <= 20")
    states = np.arange(1 << N, dtype=np.int64)
    S = 2 * ((states[:, None] >> np.arange(N, dtype=np.int64)[None, :]) & 1).astype(np.float64) - 1.0
    from oracle import exact
    pair = np.zeros(1 << N)
    for i, j in exact.bonds(L, boundary, lattice):
        pair += S[:, i] * S[:, j]
    M = S.sum(axis=1)
    E = -J * pair - H * M
    x = -beta * E
    mx = x.max()
    w = np.exp(x - mx)
    Z0 = w.sum()
    Ebar, Mbar = (w * E).sum() / Z0, (w * M).sum() / Z0
    return {"lnZ": mx + np.log(Z0), "e": Ebar / N, "c": beta * beta * ((w * E * E).sum() / Z0 - Ebar ** 2) / N,
            "m": Mbar / N, "m_abs": (w * np.abs(M)).sum() / Z0 / N,
            "chi": beta * ((w * M * M).sum() / Z0 - Mbar ** 2) / N}
