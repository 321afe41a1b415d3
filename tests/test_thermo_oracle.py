"""Pins of the thermodynamics oracle (Eq. 2 evaluated over the (k, ell) plane).

* Direct enumeration of the spin Hamiltonian (Eq. 1) over all 2^16 states of
  the 4 x 4 torus must give the same ln Z and moments as Eq. 2 evaluated on
  the brute-force degeneracies: pins the map from (k, ell) to E and M.
* J = 0 leaves independent spins in a field: Z = (2 cosh beta H)^N,
  m = tanh(beta H), chi = beta (1 - m^2), e = -H m, c = (beta H)^2 (1 - m^2).
* beta = 0 counts all states: ln Z = N ln 2, e = m = 0, c = 0, and
  chi = 0 at beta = 0 (the beta factor).
* H -> -H mirrors the magnetisation and keeps ln Z.
* The centre entropy reads the (N_B/2, N/2) entry.
"""
import math

import numpy as np
import pytest

from oracle import exact, thermo


@pytest.fixture(scope="module")
def lng4():
    return thermo.lng_from_counts(exact.brute_force(4))


@pytest.mark.parametrize("beta,H,J", [(0.1, 0.0, 1.0), (0.44, 0.0, 1.0), (0.3, 0.2, 1.0), (0.7, -0.5, 1.0),
                                      (1.5, 0.05, 1.0), (0.25, 1.0, -1.0)])
def test_eq2_equals_spin_enumeration_L4(lng4, beta, H, J):
    got = thermo.thermo(4, lng4, beta, H, J)
    ref = thermo.spin_enumeration(4, beta, H, J)
    for f in thermo.FIELDS:
        assert got[f] == pytest.approx(ref[f], rel=1e-11, abs=1e-12), f


@pytest.mark.parametrize("L", [4, 6, 8])
@pytest.mark.parametrize("beta,H", [(0.3, 0.4), (1.1, -0.25), (2.0, 0.01)])
def test_independent_spins_J0(L, beta, H):
    g = exact.transfer_matrix(L) if L > 4 else exact.brute_force(4)
    lng = thermo.lng_from_counts(np.asarray(g, dtype=np.int64))
    N = L * L
    got = thermo.thermo(L, lng, beta, H, J=0.0)
    m = math.tanh(beta * H)
    assert got["lnZ"] == pytest.approx(N * math.log(2.0 * math.cosh(beta * H)), rel=1e-12)
    assert got["m"] == pytest.approx(m, rel=1e-10, abs=1e-13)
    assert got["chi"] == pytest.approx(beta * (1.0 - m * m), rel=1e-9)
    assert got["e"] == pytest.approx(-H * m, rel=1e-10, abs=1e-13)
    assert got["c"] == pytest.approx((beta * H) ** 2 * (1.0 - m * m), rel=1e-8, abs=1e-13)


def test_infinite_temperature(lng4):
    got = thermo.thermo(4, lng4, 0.0, 0.3, 1.0)
    assert got["lnZ"] == pytest.approx(16 * math.log(2.0), rel=1e-14)
    assert abs(got["e"]) < 1e-14 and abs(got["m"]) < 1e-14
    assert got["c"] == 0.0 and got["chi"] == 0.0
    # <|M|> over all states: sum_ell C(16, ell) |2 ell - 16| / 2^16 / 16
    ref = sum(math.comb(16, e) * abs(2 * e - 16) for e in range(17)) / 2 ** 16 / 16
    assert got["m_abs"] == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("beta,H", [(0.3, 0.2), (0.6, 0.9)])
def test_field_reversal(lng4, beta, H):
    a, b = thermo.thermo(4, lng4, beta, H), thermo.thermo(4, lng4, beta, -H)
    assert a["lnZ"] == pytest.approx(b["lnZ"], rel=1e-14)
    assert a["m"] == pytest.approx(-b["m"], rel=1e-12)
    for f in ("e", "c", "m_abs", "chi"):
        assert a[f] == pytest.approx(b[f], rel=1e-11), f


def test_center_entropy(lng4):
    bf = exact.brute_force(4)
    assert thermo.center_entropy(4, lng4) == pytest.approx(math.log(bf[8, 16]) / 16, rel=1e-15)
    assert bf[8, 16] > 0


def test_planted_sign_error_is_caught(lng4):
    """A flipped field term (the sign printed in Eq. 2 with ell counting up
    spins) must fail the enumeration pin: evaluating at -H is the same
    mistake, and it reverses the magnetisation."""
    beta, H = 0.5, 0.3
    ref = thermo.spin_enumeration(4, beta, H)
    wrong = thermo.thermo(4, lng4, beta, -H)       # same as flipping the sign of the field term
    assert wrong["m"] == pytest.approx(-ref["m"], rel=1e-12) and abs(ref["m"]) > 0.1
