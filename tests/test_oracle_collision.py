"""Pins of the oracle's equilibrium and BGK collision.

* Sec. 2 (rule of Nie et al.): a rule of degree d >= N + M reproduces moments
  of order M exactly; with M <= N <= d/2 the discrete moments of the truncated
  Hermite equilibrium (App. A) are therefore exactly the moments of the
  Maxwellian of density rho, velocity u and temperature theta T0, i.e. of a
  Gaussian with mean u and variance theta c_s^2 per axis (T0 = c_s^2).  The
  tests write those Gaussian moments in closed form.
* Sec. 3: density and momentum (and, in the compressible model, the energy
  2 rho C_v theta) are collision invariants, and f = f^eq is a fixed point.
* Sec. 3: in the compressible model tau = mu/(c_s^2 dt P) + 1/2 with constant
  mu, so (tau - 1/2) P is the same in every cell, P = rho theta.
"""
import itertools
import math

import numpy as np
import pytest

VALID = [(s, N) for s, d in [("D2Q9", 5), ("D2Q19", 9), ("D2Q25", 9), ("D3Q13", 5), ("D3Q21", 5),
                             ("D3Q27", 5), ("D3V27", 7), ("D3Q45", 9)] for N in range(2, d // 2 + 1)]


def dfact(k):
    return 1 if k <= 0 else k * dfact(k - 2)


def gauss1d(u, sig2, k):
    """E[(u + sigma Z)^k] for a standard normal Z."""
    return sum(math.comb(k, j) * u ** (k - j) * sig2 ** (j / 2) * dfact(j - 1) for j in range(0, k + 1, 2))


def maxwell_moment(rho, u, sig2, p):
    out = rho
    for a, k in enumerate(p):
        out *= gauss1d(u[a], sig2, k)
    return out


def scaled_xi(orc, name, cs):
    t = orc.table(name)
    return t["xi"] * (cs / t["cs"]), t


@pytest.mark.parametrize("name,N", VALID)
def test_equilibrium_moments_are_maxwellian(orc, name, N):
    D = orc.table(name)["D"]
    cs = 0.8  # any c_s: the set is rescaled (Sec. 2) and T0 = c_s^2
    compressible = N == 4
    cfg = orc.Config(name, (1, 1, 1), tau=1.0, order=N, stencil=1, cs=cs, compressible=compressible)
    xi, _ = scaled_xi(orc, name, cs)
    rng = np.random.default_rng(N + 10 * D)
    for theta in ([1.0] if not compressible else [0.7, 1.0, 1.3]):
        rho = 1.0 + rng.uniform(-0.2, 0.2)
        u = rng.uniform(-0.3, 0.3, size=3) * cs
        feq = orc.feq(cfg, rho, u[:D], theta)
        f = feq[:cfg.Q]
        for M in range(N + 1):
            for p in itertools.product(range(M + 1), repeat=D):
                if sum(p) != M:
                    continue
                got = float(np.sum(f * np.prod(xi ** np.array(p), axis=1)))
                exp = maxwell_moment(rho, u[:D], theta * cs * cs, p)
                scale = float(np.sum(np.abs(f) * np.abs(np.prod(xi ** np.array(p), axis=1))))
                assert abs(got - exp) <= 1e-12 * max(scale, 1.0), (name, N, theta, p, got, exp)
        if compressible:
            g = feq[cfg.Q:]
            Cv = 1.0 / (1.4 - 1.0)
            # g^eq = theta (2 C_v - D) f^eq (Sec. 3) carries rho theta (2 C_v - D)
            assert np.sum(g) == pytest.approx(theta * (2 * Cv - D) * rho, rel=1e-13)


@pytest.mark.parametrize("name,N", VALID)
def test_equilibrium_is_a_fixed_point(orc, name, N):
    compressible = N == 4
    cfg = orc.Config(name, (1, 1, 1), tau=0.73, order=N, stencil=1, compressible=compressible)
    D = cfg.D
    cs = orc.table(name)["cs"]
    u = np.array([0.11, -0.07, 0.05])[:D] * cs
    feq = orc.feq(cfg, 1.03, u, 1.1 if compressible else 1.0)
    out = orc.collide_one(cfg, feq)
    assert np.max(np.abs(out - feq)) <= 1e-14 * np.max(np.abs(feq))


@pytest.mark.parametrize("name,N", VALID)
def test_collision_conserves_invariants(orc, name, N):
    compressible = N == 4
    cfg = orc.Config(name, (1, 1, 1), tau=0.61, order=N, stencil=1, compressible=compressible)
    cs = orc.table(name)["cs"]
    xi, t = scaled_xi(orc, name, cs)
    rng = np.random.default_rng(7)
    base = orc.feq(cfg, 1.0, np.array([0.05, -0.02, 0.03])[:cfg.D] * cs, 1.0)
    f = base * (1.0 + rng.uniform(-0.05, 0.05, size=base.shape))
    out = orc.collide_one(cfg, f)
    Q = cfg.Q
    for a, b in [(f, out)]:
        assert np.sum(b[:Q]) == pytest.approx(np.sum(a[:Q]), rel=1e-14)
        for ax in range(cfg.D):
            assert np.sum(xi[:, ax] * b[:Q]) == pytest.approx(np.sum(xi[:, ax] * a[:Q]), abs=1e-14 * cs)
        if compressible:
            # total energy sum(|xi|^2 f / T0 + g) = 2 rho C_v theta + rho |u|^2 / T0
            x2 = np.sum(xi * xi, axis=1) / cs ** 2
            e_a = np.sum(x2 * a[:Q]) + np.sum(a[Q:])
            e_b = np.sum(x2 * b[:Q]) + np.sum(b[Q:])
            assert e_b == pytest.approx(e_a, rel=1e-13)


@pytest.mark.parametrize("name", ["D2Q19", "D2Q25", "D3Q45"])
def test_temperature_round_trip(orc, name):
    """theta recovered from (f^eq, g^eq) through 2 rho C_v theta = sum(|zeta|^2 f/T0 + g)."""
    cs = 0.8  # T0 = c_s^2 differs from 1
    cfg = orc.Config(name, (1, 1, 1), tau=1.0, order=4, stencil=1, compressible=True, gamma=1.4, cs=cs)
    for theta in (0.6, 1.0, 1.45):
        rho = 0.9
        u = np.array([0.2, -0.1, 0.15])[:cfg.D] * cs
        f = orc.feq(cfg, rho, u, theta).reshape((cfg.A * cfg.Q, 1, 1, 1))
        r, uu, th, _ = orc.moments(cfg, f)
        assert r.item() == pytest.approx(rho, rel=1e-14)
        assert np.allclose(uu.ravel(), u, rtol=0, atol=1e-14)
        assert th.item() == pytest.approx(theta, rel=1e-13)


def test_pressure_dependent_relaxation(orc):
    """(tau(x) - 1/2) rho theta = tau_ref - 1/2 in every cell (Sec. 3, constant mu)."""
    name = "D2Q25"
    tau_ref = 0.9
    cfg = orc.Config(name, (1, 1, 1), tau=tau_ref, order=4, stencil=1, compressible=True, gamma=1.4)
    cs = orc.table(name)["cs"]
    rng = np.random.default_rng(3)
    for rho, theta in [(1.0, 1.0), (1.3, 0.8), (0.7, 1.4)]:
        feq = orc.feq(cfg, rho, np.array([0.1, 0.05]) * cs, theta)
        f = feq * (1.0 + rng.uniform(-0.02, 0.02, size=feq.shape))
        # the collision relaxes towards the equilibrium of f's own moments
        r, uu, th, _ = orc.moments(cfg, f.reshape((-1, 1, 1, 1)))
        feq_f = orc.feq(cfg, r.item(), uu.ravel(), th.item())
        out = orc.collide_one(cfg, f)
        k = np.argmax(np.abs(f - feq_f))
        factor = (out[k] - feq_f[k]) / (f[k] - feq_f[k])  # = 1 - 1/tau(x)
        tau_x = 1.0 / (1.0 - factor)
        assert (tau_x - 0.5) * r.item() * th.item() == pytest.approx(tau_ref - 0.5, rel=1e-9)
