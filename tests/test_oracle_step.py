"""Pins of whole oracle time steps (stream, then collide; Sec. 3).

* Periodic steps conserve mass and momentum (and, in the compressible model,
  total energy): streaming conserves each population's sum, collision the
  moments (Sec. 3, eqs. density, momentum, and the temperature definition).
* The 2D Taylor-Green vortex decays as exp(-2 nu k^2 t) with the viscosity
  nu = c_s^2 (tau - 1/2) dt of Sec. 3, within the interpolation's own
  numerical dissipation (about 1 % of the rate at 64^2 with the three-point
  stencil), and the error shrinks under refinement.
* A uniform state at equilibrium stays put.
"""
import math

import numpy as np
import pytest

import lbm_inputs as W


def smooth_fields(D, shape, amp, seed):
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(s) * 2 * math.pi / s for s in shape], indexing="ij")
    u = []
    for a in range(D):
        ph = rng.uniform(0, 2 * math.pi, size=3)
        u.append(amp * np.sin(grids[2] + ph[0]) * np.cos(grids[1] + ph[1]) * np.cos(grids[0] + ph[2]))
    rho = 1.0 + 0.01 * np.cos(grids[2] + grids[1])
    return rho, np.stack(u)


@pytest.mark.parametrize("name,N,compressible", [("D2Q9", 2, False), ("D3Q13", 2, False), ("D3V27", 3, False),
                                                 ("D2Q25", 4, True), ("D3Q45", 4, True)])
def test_periodic_steps_conserve(orc, name, N, compressible):
    D = orc.table(name)["D"]
    cs = orc.table(name)["cs"]
    grid = (8, 7, 6) if D == 3 else (12, 10, 1)
    cfg = orc.Config(name, grid, tau=0.7, order=N, stencil=4, dx=1.0, dt=0.35 / cs, cs=cs,
                     compressible=compressible)
    rho, u = smooth_fields(D, cfg.shape, 0.1 * cs, 1)
    theta = 1.0 + 0.05 * np.cos(np.arange(cfg.ncell).reshape(cfg.shape)) if compressible else None
    f = orc.init(cfg, rho, u, theta)
    _, _, _, d0 = orc.moments(cfg, f)
    f = orc.run(cfg, f, 3)
    _, _, _, d1 = orc.moments(cfg, f)
    assert d1["mass"] == pytest.approx(d0["mass"], rel=1e-13)
    assert np.allclose(d1["momentum"], d0["momentum"], rtol=0, atol=1e-13 * d0["mass"] * cs)
    if compressible:
        assert d1["energy"] == pytest.approx(d0["energy"], rel=1e-12)


def test_uniform_equilibrium_is_steady(orc):
    cfg = orc.Config("D3Q21", (6, 5, 4), tau=0.55, order=2, stencil=4, dx=1.0, dt=0.3)
    cs = orc.table("D3Q21")["cs"]
    rho = np.full(cfg.shape, 1.02)
    u = np.zeros((3,) + cfg.shape)
    u[0] = 0.05 * cs
    u[2] = -0.02 * cs
    f = orc.init(cfg, rho, u)
    g = orc.run(cfg, f, 2)
    assert np.max(np.abs(g - f)) <= 1e-14


def tgv_amplitude(u, wl):
    nx = wl.grid[0]
    k = 2 * math.pi / nx
    j = np.arange(nx)
    X, Y = np.meshgrid(j, j, indexing="xy")
    mode = np.sin(k * X) * np.cos(k * Y)
    return float(np.sum(u[0, 0] * mode) / np.sum(mode * mode))


def _tgv_run(orc, n, steps):
    wl = W.tgv2d_workload(n=n, steps=steps)
    cfg = orc.Config(wl.set, wl.grid, tau=wl.tau, order=wl.order, stencil=wl.stencil, dx=wl.dx, dt=wl.dt,
                     cs=wl.cs)
    rho, u, _ = W.tgv2d_fields(wl, noise=0.0)
    f0 = orc.init(cfg, rho, u)
    _, u0, _, _ = orc.moments(cfg, f0)
    f = orc.run(cfg, f0, steps)
    _, u1, _, _ = orc.moments(cfg, f)
    ratio = tgv_amplitude(u1, wl) / tgv_amplitude(u0, wl)
    return ratio, W.tgv2d_decay(wl, steps * wl.dt)


def test_tgv2d_viscous_decay(orc):
    """64^2, 1000 steps: decay rate within 2 % of that of exp(-2 nu k^2 t)."""
    ratio, exact = _tgv_run(orc, 64, 1000)
    rate, rate_exact = -math.log(ratio), -math.log(exact)
    assert abs(rate / rate_exact - 1.0) < 0.02, (ratio, exact)


@pytest.mark.slow
def test_tgv2d_refinement(orc):
    """Doubling the resolution (same Re, same physical time) shrinks the error."""
    r64, e64 = _tgv_run(orc, 32, 250)
    r128, e128 = _tgv_run(orc, 64, 1000)  # dt fixed at 0.5: 4x the steps for 2x n (diffusive scaling)
    err64 = abs(math.log(r64) / math.log(e64) - 1)
    err128 = abs(math.log(r128) / math.log(e128) - 1)
    assert err128 < err64
