"""Pins of the oracle's diagnostics and of its one-step-at-selected-cells
evaluation (CPU only).

* Kinetic energy k = <|u|^2/2> over the nodes, without density weighting
  (Sec. 4.2): the 3D Taylor-Green field of Sec. 4.2 (u0 = 1) has k = 1/8 and
  the 2D one u0^2/4 on any uniform periodic grid with at least three nodes
  per axis (the node mean of sin^2 and cos^2 is exactly 1/2 there).
* Smallest density and temperature: a planted minimum is found, and the
  per-cell fields of an equilibrium state give back the fields it was built
  from (the equilibrium's density, momentum and temperature moments are
  exact for every set and order used, Sec. 2).
* Mass, momentum and the total energy moment against their closed forms:
  for f = f^eq (and g = g^eq), sum_i |xi_i|^2 f_i / T0 + g_i =
  rho |u|^2 / T0 + 2 C_v rho theta (the Maxwellian's second moment
  rho (u u + theta T0 I) and g^eq = theta (2 C_v - D) f^eq, Sec. 3).
* One step evaluated at selected cells (``first_step_at``, the reference of
  the full-size sampled GPU tests) equals the whole-grid step of the
  equilibrium state at those cells: grid corners, tile edges, both arrays of
  the compressible model, and extrapolating axes.
"""
import math

import numpy as np
import pytest

import lbm_inputs as W


def axes(shape):
    """Node coordinates 2 pi j / n of a [nz][ny][nx] grid, as (z, y, x)."""
    return np.meshgrid(*[np.arange(s) * 2 * math.pi / s for s in shape], indexing="ij")


@pytest.mark.parametrize("name,N,n", [("D3Q27", 2, 16), ("D3Q13", 2, 9), ("D3V27", 3, 12)])
def test_ke_of_3d_taylor_green_is_one_eighth(orc, name, N, n):
    cs = 10.0
    cfg = orc.Config(name, (n, n, n), tau=0.6, order=N, stencil=4, dx=2 * math.pi / n, dt=1e-3, cs=cs)
    z, y, x = axes(cfg.shape)
    u = np.stack([np.sin(x) * np.cos(y) * np.cos(z), -np.cos(x) * np.sin(y) * np.cos(z), 0.0 * x])
    rho = 1.0 + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / (16 * cs * cs)
    _, _, _, d = orc.moments(cfg, orc.init(cfg, rho, u))
    assert abs(d["ke"] / 0.125 - 1.0) <= 1e-14, d["ke"]


@pytest.mark.parametrize("n", [3, 8, 64])
def test_ke_of_2d_taylor_green(orc, n):
    cs = 1.0 / math.sqrt(3.0)
    u0 = 0.05 * cs
    cfg = orc.Config("D2Q9", (n, n, 1), tau=0.6, order=2, stencil=3, dx=1.0, dt=0.5, cs=cs)
    _, y, x = axes(cfg.shape)
    u = u0 * np.stack([np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)])
    rho = 1.0 + u0 * u0 / (4 * cs * cs) * (np.cos(2 * x) + np.cos(2 * y))
    _, _, _, d = orc.moments(cfg, orc.init(cfg, rho, u))
    assert abs(d["ke"] / (u0 * u0 / 4) - 1.0) <= 1e-13, d["ke"]


def test_ke_of_compressible_taylor_green(orc):
    """The compressible model (f and g, theta != 1) gives the same k."""
    wl = W.ctgv_workload(n=8, Ma=1.0)
    cfg = orc.Config("D3Q45", wl.grid, tau=wl.tau, order=4, stencil=4, dx=wl.dx, dt=wl.dt, cs=wl.cs,
                     compressible=True, gamma=wl.gamma)
    rho, u, theta = W.ctgv_fields(wl)
    theta = theta * (1.0 + 0.1 * np.cos(axes(cfg.shape)[0]))
    _, _, _, d = orc.moments(cfg, orc.init(cfg, rho, u, theta))
    assert abs(d["ke"] / 0.125 - 1.0) <= 1e-13, d["ke"]


@pytest.mark.parametrize("name,N,comp", [("D3Q21", 2, False), ("D2Q25", 4, True), ("D3Q45", 4, True)])
def test_diagnostics_closed_forms(orc, name, N, comp):
    t = orc.table(name)
    D, cs = t["D"], 0.8 * t["cs"]
    grid = (7, 6, 5) if D == 3 else (9, 8, 1)
    gamma = 1.4
    cfg = orc.Config(name, grid, tau=0.7, order=N, stencil=4, dx=1.0, dt=0.2, cs=cs, compressible=comp,
                     gamma=gamma)
    rng = np.random.default_rng(3)
    rho = rng.uniform(0.95, 1.05, cfg.shape)
    u = rng.uniform(-0.2 * cs, 0.2 * cs, (D,) + cfg.shape)
    theta = rng.uniform(0.9, 1.1, cfg.shape) if comp else np.ones(cfg.shape)
    flat = np.unravel_index(17, cfg.shape)
    rho[flat] = 0.8125            # planted minima, at different cells
    theta[np.unravel_index(5, cfg.shape)] = 0.6875 if comp else 1.0
    f = orc.init(cfg, rho, u, theta if comp else None)
    r, uu, th, d = orc.moments(cfg, f)
    # per-cell fields give back the fields the equilibrium was built from
    assert np.max(np.abs(r - rho)) <= 1e-14
    assert np.max(np.abs(uu - u)) <= 1e-14 * cs
    assert np.max(np.abs(th - theta)) <= 1e-13
    assert abs(d["min_rho"] - 0.8125) <= 1e-15
    assert abs(d["min_theta"] - (0.6875 if comp else 1.0)) <= 1e-13
    assert abs(d["mass"] / rho.sum() - 1.0) <= 1e-14
    mom = (rho * u).reshape(D, -1).sum(axis=1)
    assert np.max(np.abs(d["momentum"] - mom)) <= 1e-14 * rho.sum() * cs
    u2 = np.sum(u * u, axis=0)
    Cv = 1.0 / (gamma - 1.0) if comp else 0.5 * D
    energy = 0.5 * np.sum(rho * u2 / (cs * cs) + 2.0 * Cv * rho * theta)
    assert abs(d["energy"] / energy - 1.0) <= 1e-13, (d["energy"], energy)
    assert abs(d["ke"] / np.mean(0.5 * u2) - 1.0) <= 1e-13


CASES = {
    # (set, grid, order, stencil, compressible, boundary, dt in cells of the fastest component)
    "d3q27_periodic": ("D3Q27", (70, 9, 6), 2, 4, False, (0, 0, 0), 0.45),
    "d3v27_large_shift": ("D3V27", (66, 10, 12), 3, 4, False, (0, 0, 0), 2.6),
    "d3q45_f_and_g": ("D3Q45", (66, 9, 8), 4, 4, True, (0, 0, 0), 0.8),
    "d2q19_clamped_x": ("D2Q19", (70, 21, 1), 4, 5, True, (1, 0, 0), 0.6),
    "d3q21_clamped_y_z": ("D3Q21", (66, 9, 7), 2, 3, False, (0, 1, 1), 0.7),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_first_step_at_equals_whole_grid_step(orc, case):
    name, grid, N, n, comp, bc, cells = CASES[case]
    t = orc.table(name)
    D, cs = t["D"], 0.6
    dt = cells / (W.MAX_COMPONENT_OVER_CS[name] * cs)
    cfg = orc.Config(name, grid, tau=0.58, order=N, stencil=n, dx=1.0, dt=dt, cs=cs, compressible=comp,
                     bc=bc)
    rho, u, theta = W.random_fields(D, cfg.shape, 9, u_amp=0.1 * cs, rho_amp=0.03,
                                    theta_amp=0.05 if comp else 0.0)
    th = theta if comp else None
    whole = orc.run(cfg, orc.init(cfg, rho, u, th), 1).reshape(cfg.A * cfg.Q, -1)
    nx, ny = grid[0], grid[1]
    picks = [0, cfg.ncell - 1, nx - 1, 63, 64, nx * (ny - 1), nx * ny - 1, cfg.ncell - nx]
    picks += list(np.random.default_rng(10).choice(cfg.ncell, 24, replace=False))
    picks = np.array(sorted(set(int(c) for c in picks)))
    got = orc.first_step_at(cfg, rho, u, picks, theta=th)
    ref = whole[:, picks].T
    assert np.max(np.abs(got - ref)) <= 1e-15 * np.max(np.abs(ref)), float(np.max(np.abs(got - ref)))
