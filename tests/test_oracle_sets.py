"""Pins of the oracle's velocity sets against what the paper fixes.

Sec. 2 defines the degree d of a rule as the largest total degree of monomials
it integrates exactly against omega(xi) = (2 pi)^{-D/2} exp(-|xi|^2/2); App. B
lists the resulting symmetry conditions (sum w = 1, sum w xi xi = c_s^2 delta,
..., c_s^8 Delta_8).  With the scale c_s those moments are the moments of a
Gaussian of variance c_s^2 per axis, which the tests write in closed form
((k-1)!! c_s^k for even k, 0 for odd k) without using any oracle code.
"""
import itertools
import math

import numpy as np
import pytest

SETS = ["D2Q9", "D2Q19", "D2Q25", "D3Q13", "D3Q21", "D3Q27", "D3V27", "D3Q45"]
EXPECTED = {  # (Q, D, degree) from Table tab:sets and the names
    "D2Q9": (9, 2, 5), "D2Q19": (19, 2, 9), "D2Q25": (25, 2, 9), "D3Q13": (13, 3, 5),
    "D3Q21": (21, 3, 5), "D3Q27": (27, 3, 5), "D3V27": (27, 3, 7), "D3Q45": (45, 3, 9),
}
# printed digits reach ~3e-13 in the D3Q45 moments (App. E); all others <= 2e-14
TOL = {"D3Q45": 1e-12}


def dfact(k):
    return 1 if k <= 0 else k * dfact(k - 2)


def gauss_moment(powers, cs):
    out = 1.0
    for k in powers:
        out *= 0.0 if k % 2 else dfact(k - 1) * cs ** k
    return out


def monomials(D, deg):
    for p in itertools.product(range(deg + 1), repeat=D):
        if sum(p) == deg:
            yield p


def moment(t, p):
    return float(np.sum(t["w"] * np.prod(t["xi"] ** np.array(p), axis=1)))


def abs_moment(t, p):
    """Scale of the sum's rounding error: sum w |prod xi^p|."""
    return float(np.sum(t["w"] * np.abs(np.prod(t["xi"] ** np.array(p), axis=1))))


@pytest.mark.parametrize("name", SETS)
def test_shape_and_degree(orc, name):
    t = orc.table(name)
    assert (t["Q"], t["D"], t["degree"]) == EXPECTED[name]
    assert t["w"].min() > 0


@pytest.mark.parametrize("name", SETS)
def test_exact_up_to_degree(orc, name):
    """Every monomial of total degree <= d is integrated exactly (Sec. 2)."""
    t = orc.table(name)
    tol = TOL.get(name, 2e-14)
    for deg in range(t["degree"] + 1):
        for p in monomials(t["D"], deg):
            exact = gauss_moment(p, t["cs"])
            got = moment(t, p)
            assert abs(got - exact) <= tol * max(1.0, abs_moment(t, p)), (name, p, got, exact)


@pytest.mark.parametrize("name", SETS)
def test_not_exact_at_next_even_degree(orc, name):
    """The degree is the largest one: some monomial of degree d+1 fails."""
    t = orc.table(name)
    deg = t["degree"] + 1
    worst = max(abs(moment(t, p) - gauss_moment(p, t["cs"])) / max(1.0, gauss_moment(p, t["cs"]))
                for p in monomials(t["D"], deg))
    assert worst > 1e-3


@pytest.mark.parametrize("name", SETS)
def test_central_symmetry(orc, name):
    """All eight sets contain -xi with every xi, with the same weight."""
    t = orc.table(name)
    for i in range(t["Q"]):
        j = np.where(np.all(np.abs(t["xi"] + t["xi"][i]) < 1e-15, axis=1))[0]
        assert j.size == 1 and t["w"][j[0]] == t["w"][i]


def test_printed_closed_forms(orc):
    """Closed forms stated in the table captions (Tables tab:d3q13, tab:d3q21)
    and the Gauss-Hermite roots of the product sets."""
    t13 = orc.table("D3Q13")
    r, s = math.sqrt((5 + math.sqrt(5)) / 2), math.sqrt((5 - math.sqrt(5)) / 2)
    mags = np.abs(t13["xi"]).ravel()
    for m in mags:
        assert min(abs(m - 0.0), abs(m - s), abs(m - r)) <= 1e-15
    assert t13["w"][0] == pytest.approx(2 / 5, abs=1e-16)
    assert np.allclose(t13["w"][1:], 1 / 20, atol=1e-17)
    t21 = orc.table("D3Q21")
    assert t21["cs"] == pytest.approx(math.sqrt(3 / 5), abs=1e-16)
    assert np.allclose(t21["w"][1:], 3 / 100, atol=1e-17)
    # D2Q25: roots of He_5(x) = x^5 - 10 x^3 + 15 x
    t25 = orc.table("D2Q25")
    nodes = sorted(set(np.round(t25["xi"][:, 0], 13)))
    assert np.allclose(np.polyval([1, 0, -10, 0, 15, 0], nodes), 0, atol=1e-11)
    assert len(nodes) == 5
    # D2Q9 / D3Q27 in lattice units: nodes 0, +-1 and c_s^2 = 1/3
    for name in ("D2Q9", "D3Q27"):
        t = orc.table(name)
        assert set(np.unique(t["xi"])) == {-1.0, 0.0, 1.0}
        assert t["cs"] ** 2 == pytest.approx(1 / 3, abs=4e-16)


def test_d3q45_printed_rows_are_verbatim(orc):
    """Spot check of App. E rows, typed from the paper into this test."""
    t = orc.table("D3Q45")
    assert t["w"][0] == 0.20740740740740618
    assert tuple(t["xi"][1]) == (0.06386083877343968, -1.2239121278243665, -1.2239121278243665)
    assert tuple(t["xi"][31]) == (1.7320508075688787, 1.7320508075688787, 1.7320508075688787)
    assert t["w"][44] == 0.0004629629629629939
    assert tuple(t["xi"][44]) == (-1.1335992635264445, -1.1335992635264445, 3.5256070994177073)
