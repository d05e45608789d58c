"""Pins of the oracle's flow diagnostics (``oracle/diagnostics.py``, Sec. 4.2).

* Central-difference weights: the published values for orders 2-8 (Fornberg's
  table), polynomial exactness to degree 2m and failure at 2m + 1.
* Enstrophy of the Taylor-Green velocity of Sec. 4.2: 3/4 in the continuum
  (closed form; the spectral derivative reproduces it to rounding) and
  exactly 3/4 kappa^2 with central differences, kappa being the difference
  operator's symbol at wavenumber one.
* <|curl u|^2> = <|grad u|^2> - <(div u)^2> on a periodic grid: catches a
  wrong sign, index or pairing inside a vorticity component.
* Convergence to the spectral enstrophy at the order of the differences.
"""
import math

import numpy as np
import pytest

from oracle import diagnostics as G

FORNBERG = {
    1: [1 / 2],
    2: [2 / 3, -1 / 12],
    3: [3 / 4, -3 / 20, 1 / 60],
    4: [4 / 5, -1 / 5, 4 / 105, -1 / 280],
}


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_weights_match_published_table(m):
    assert np.allclose(G.central_difference_weights(m), FORNBERG[m], rtol=1e-13, atol=0)


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_weights_exact_to_degree_2m(m):
    h = 0.1
    x = np.arange(40) * h
    inner = slice(m, 40 - m)
    for deg in range(0, 2 * m + 2):
        f = (x - 1.3) ** deg
        exact = deg * (x - 1.3) ** (deg - 1) if deg > 0 else np.zeros_like(x)
        got = G.derivative(f.reshape(1, 1, -1), 0, h, 2 * m)[0, 0]
        err = np.max(np.abs(got[inner] - exact[inner]))
        if deg <= 2 * m:
            assert err < 1e-9 * max(1.0, np.max(np.abs(exact))), (m, deg, err)
        else:
            assert err > 1e-6, (m, deg, err)


def tgv_velocity(n):
    x = np.arange(n) * 2 * math.pi / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    return np.stack([np.sin(X) * np.cos(Y) * np.cos(Z), -np.cos(X) * np.sin(Y) * np.cos(Z), np.zeros_like(X)])


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_tgv_enstrophy_closed_form(order):
    n = 24
    dx = 2 * math.pi / n
    u = tgv_velocity(n)
    # curl of the Sec. 4.2 field: (-cos x sin y sin z, -sin x cos y sin z, 2 sin x sin y cos z),
    # mean square 1/8 + 1/8 + 4/8 = 3/4; every derivative acts on a wavenumber-one mode,
    # which the differences scale by kappa = sum_j 2 a_j sin(j dx) / dx
    a = G.central_difference_weights(order // 2)
    kappa = sum(2 * aj * math.sin(j * dx) for j, aj in enumerate(a, start=1)) / dx
    assert G.enstrophy(u, dx, order) == pytest.approx(0.75 * kappa ** 2, rel=1e-13)
    assert abs(0.75 * kappa ** 2 - 0.75) < 2 * dx ** order
    assert G.spectral_enstrophy(u, dx) == pytest.approx(0.75, rel=1e-13)
    assert G.kinetic_energy(u) == pytest.approx(0.125, rel=1e-13)


def smooth_field(D, n, seed, kmax=3):
    rng = np.random.default_rng(seed)
    x = np.arange(n) * 2 * math.pi / n
    shape = (n, n, n) if D == 3 else (1, n, n)
    grids = np.meshgrid(*([x] * 3 if D == 3 else [np.zeros(1), x, x]), indexing="ij")
    Z, Y, X = grids
    u = np.zeros((D,) + shape)
    # every component over one set of wavevectors, so that products of
    # different components' derivatives have non-zero means
    for _ in range(8):
        k = rng.integers(-kmax, kmax + 1, size=3)
        if D == 2:
            k[0] = 0
        for c in range(D):
            ph = rng.uniform(0, 2 * math.pi)
            u[c] += rng.normal() * np.cos(k[2] * X + k[1] * Y + k[0] * Z + ph)
    return u


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("order", [2, 8])
def test_curl_identity(D, order):
    n = 20
    dx = 2 * math.pi / n
    u = smooth_field(D, n, seed=D) + 0.1 * np.random.default_rng(9).normal(size=(D,) + ((n,) * 3 if D == 3 else (1, n, n)))
    grad2, div2 = G.gradient_norms(u, dx, order)
    assert G.enstrophy(u, dx, order) == pytest.approx(grad2 - div2, rel=1e-12)


def test_curl_identity_catches_wrong_components():
    n = 16
    dx = 2 * math.pi / n
    u = smooth_field(3, n, seed=4)
    grad2, div2 = G.gradient_norms(u, dx, 4)
    good = G.enstrophy(u, dx, 4)
    assert good == pytest.approx(grad2 - div2, rel=1e-12)
    d = lambda c, a: G.derivative(u[c], a, dx, 4)  # noqa: E731
    wrong = [
        np.stack([d(2, 1) + d(1, 2), d(0, 2) - d(2, 0), d(1, 0) - d(0, 1)]),  # sign inside a component
        np.stack([d(2, 2) - d(1, 1), d(0, 2) - d(2, 0), d(1, 0) - d(0, 1)]),  # derivative along the wrong axis
        np.stack([d(2, 1) - d(1, 2), d(0, 2) - d(2, 0), d(1, 1) - d(0, 0)]),  # components paired wrongly
    ]
    for w in wrong:
        bad = float(np.mean(np.sum(w * w, axis=0)))
        assert abs(bad / (grad2 - div2) - 1) > 1e-3


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("order", [2, 4, 6])
def test_converges_to_spectral_at_its_order(D, order):
    errs = []
    for n in (16, 32):
        u = smooth_field(D, n, seed=11)
        dx = 2 * math.pi / n
        errs.append(abs(G.enstrophy(u, dx, order) - G.spectral_enstrophy(u, dx)))
    assert errs[0] / errs[1] > 0.6 * 2 ** order, errs
