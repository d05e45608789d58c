"""Pins of the oracle's cell-wise streaming on Gauss-Lobatto-Chebyshev support
points (the paper's own discretization, Sec. 3, eq. sl_streaming): every axis
is divided into cells of p + 1 support points at the extrema of the
Chebyshev polynomial T_p mapped onto the cell, neighbouring cells sharing
their end points; each node's departure point is interpolated with the
polynomial of the cell that holds it.

* A hand-worked example with p = 2 (tests/golden/glc_p2_quarter_cell.txt).
* Polynomial exactness: a field that is a polynomial of degree <= p along
  each axis, sampled at the Gauss-Lobatto-Chebyshev node coordinates, is
  interpolated exactly at the departure points (p = 4, 2D and 3D, shifts of
  a fraction of a cell and of more than one cell).  Sampling the same field
  at uniform coordinates instead would break it, so this pins the support
  points themselves.
* Convergence at order p + 1 for a smooth periodic field: halving the cell
  width shrinks the error by at least 2^p.
* No shift is the identity, bit for bit; a shift of exactly one cell is a
  shift of the array by p nodes.
Unlike the uniform stencil, cell-wise streaming does not conserve the node
sum of a population (the phase of a node within its cell changes its
weights), so conservation is not a pin here.
"""
import math
import os

import numpy as np
import pytest

import lbm_inputs as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=", 1)
                out[k.strip()] = np.array([float(x) for x in v.split()])
    return out


def d2q9_plus_x(orc):
    """Index of D2Q9's population moving +1 node per unit time along x."""
    t = orc.table("D2Q9")
    xh = t["xi"] / t["cs"]
    return int(np.flatnonzero((np.abs(xh[:, 0] - math.sqrt(3.0)) < 1e-12) & (np.abs(xh[:, 1]) < 1e-12))[0])


def test_hand_worked_p2_quarter_cell(orc):
    g = golden("glc_p2_quarter_cell.txt")
    cs = 1.0 / math.sqrt(3.0)
    # D2Q9 in lattice units (xi_x = 1 for the +x population), dt = 0.5: half a node per step
    cfg = orc.Config("D2Q9", (4, 2, 1), tau=0.8, order=2, stencil=3, dx=1.0, dt=0.5, cs=cs, kind="glc")
    i = d2q9_plus_x(orc)
    f = np.zeros(cfg.pop_shape())
    f[i, 0, :, :] = g["input"][None, :]
    out = orc.stream(cfg, f)
    # (to rounding: the support point 1/2 is (1 - cos(pi/2))/2 in floating point)
    for y in range(2):
        assert np.max(np.abs(out[i, 0, y] - g["output"])) <= 1e-14, out[i, 0, y]


def _poly(coords, degs, seed):
    """A random polynomial of degree degs[a] in coordinate a (tensor form)."""
    rng = np.random.default_rng(seed)
    val = 1.0
    for x, d in zip(coords, degs):
        c = rng.uniform(-1, 1, d + 1)
        val = val * np.polynomial.polynomial.polyval(x, c)
    return val


@pytest.mark.parametrize("name,grid,dt_cells", [("D2Q9", (24, 24, 1), 0.3), ("D2Q19", (40, 40, 1), 1.7),
                                                ("D3Q13", (24, 24, 24), 0.6)])
def test_polynomial_exactness_p4(orc, name, grid, dt_cells):
    p = 4
    D = W.DIM[name]
    cs = 1.0
    dx = 0.5
    dt = dt_cells * p * dx / (W.MAX_COMPONENT_OVER_CS[name] * cs)  # fastest component: dt_cells cells per step
    cfg = orc.Config(name, grid, tau=0.8, order=2, stencil=p + 1, dx=dx, dt=dt, cs=cs, kind="glc")
    nz, ny, nx = cfg.shape
    X = W.glc_nodes(nx, p, dx)
    Y = W.glc_nodes(ny, p, dx)
    Z = W.glc_nodes(nz, p, dx) if D == 3 else np.zeros(1)
    ZZ, YY, XX = np.meshgrid(Z, Y, X, indexing="ij")
    t = orc.table(name)
    xi = t["xi"] / t["cs"] * cs
    f = np.empty(cfg.pop_shape())
    for i in range(cfg.Q):
        f[i] = _poly((XX, YY, ZZ)[:D], (p,) * D, 40 + i)
    out = orc.stream(cfg, f)
    # nodes whose departure cell does not wrap around the periodic grid
    margin = (int(math.ceil(dt_cells)) + 1) * p
    sl = tuple(slice(margin, n - margin) if n > 1 else slice(None) for n in (nz, ny, nx))
    assert all(s.stop is None or s.stop > s.start for s in sl)
    worst = 0.0
    for i in range(cfg.Q):
        dep = [XX - xi[i, 0] * dt, YY - xi[i, 1] * dt] + ([ZZ - xi[i, 2] * dt] if D == 3 else [])
        exact = _poly(dep, (p,) * D, 40 + i)
        worst = max(worst, float(np.max(np.abs(out[i][sl] - exact[sl]) / np.max(np.abs(exact[sl])))))
    assert worst <= 1e-12, worst


def test_uniform_coordinates_would_fail(orc):
    """Control for the pin above: the same polynomial sampled at uniform
    coordinates is not reproduced, so the exactness really checks that the
    oracle interpolates on Gauss-Lobatto-Chebyshev points."""
    p, dx, dt = 4, 0.5, 0.3 * 4 * 0.5 / math.sqrt(3.0)
    cfg = orc.Config("D2Q9", (24, 16, 1), tau=0.8, order=2, stencil=p + 1, dx=dx, dt=dt, cs=1.0, kind="glc")
    i = d2q9_plus_x(orc)
    Xu = np.arange(24) * dx
    f = np.zeros(cfg.pop_shape())
    f[i, 0] = _poly((Xu,), (p,), 7)[None, :]
    out = orc.stream(cfg, f)[i, 0, 0, 10:14]
    exact = _poly((Xu[10:14] - math.sqrt(3.0) * dt,), (p,), 7)
    assert np.max(np.abs(out - exact)) > 1e-6


def test_convergence_order(orc):
    """sin(k x) along x on 8, 16 and 32 cells (p = 4): the error of one
    streaming step falls by at least 2^4 per halving of the cell width."""
    p = 4
    errs = []
    for cells in (8, 16, 32):
        n = cells * p
        dx = 2 * math.pi / n
        cs = 1.0 / math.sqrt(3.0)
        dt = 0.37 * p * dx  # xi_x = 1: 0.37 cells per step
        cfg = orc.Config("D2Q9", (n, 4, 1), tau=0.8, order=2, stencil=p + 1, dx=dx, dt=dt, cs=cs, kind="glc")
        i = d2q9_plus_x(orc)
        X = W.glc_nodes(n, p, dx)
        f = np.zeros(cfg.pop_shape())
        f[i, 0] = np.sin(X + 0.3)[None, :]
        out = orc.stream(cfg, f)[i, 0, 0]
        errs.append(float(np.max(np.abs(out - np.sin(X - dt + 0.3)))))
    assert errs[0] / errs[1] >= 2 ** p and errs[1] / errs[2] >= 2 ** p, errs


def test_no_shift_and_whole_cell_shift(orc):
    p, dx = 4, 1.0
    cs = 1.0 / math.sqrt(3.0)
    i = d2q9_plus_x(orc)
    rng = np.random.default_rng(3)
    for dt, roll in ((p * dx, p), (2 * p * dx, 2 * p)):
        cfg = orc.Config("D2Q9", (16, 8, 1), tau=0.8, order=2, stencil=p + 1, dx=dx, dt=dt, cs=cs, kind="glc")
        f = rng.uniform(0.5, 1.5, cfg.pop_shape())
        out = orc.stream(cfg, f)
        assert np.array_equal(out[0], f[0])  # the rest population does not move
        assert np.max(np.abs(out[i] - np.roll(f[i], roll, axis=2))) <= 1e-15 * np.max(np.abs(f[i]))
