"""Seeded synthetic inputs for the semi-Lagrangian lattice Boltzmann step.

This module is shared by the GPU library's callers and by the CPU oracle's
tests, and it holds none of the method's arithmetic: no streaming, moments,
equilibrium or collision.  It provides

* the parameters of each workload (grid, spacing, time step, speed of sound,
  relaxation time, stencil length, truncation order), derived from the
  dimensionless numbers of the paper's test cases (Sec. 4) with the unit
  system tau = nu / (c_s^2 dt) + 1/2 (Sec. 3);
* the analytic initial fields (density, velocity, temperature) of those test
  cases, and seeded noise;
* seeded random directions for derivative checks.

The velocity sets' largest velocity component over c_s, needed to pick a time
step for a given Courant number, is copied from the printed tables (Tables
tab:d3q13, tab:d3q21, App. C-E) as plain constants.

All arrays are float64 numpy arrays, x fastest: scalars ``[nz][ny][nx]`` and
velocities ``[D][nz][ny][nx]`` (nz = 1 in 2D).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

SETS = ("D2Q9", "D2Q19", "D2Q25", "D3Q13", "D3Q21", "D3Q27", "D3V27", "D3Q45")
DIM = {"D2Q9": 2, "D2Q19": 2, "D2Q25": 2, "D3Q13": 3, "D3Q21": 3, "D3Q27": 3, "D3V27": 3, "D3Q45": 3}
DEGREE = {"D2Q9": 5, "D2Q19": 9, "D2Q25": 9, "D3Q13": 5, "D3Q21": 5, "D3Q27": 5, "D3V27": 7, "D3Q45": 9}

# Largest |xi_{i,alpha}| / c_s of each set, from the printed tables.
MAX_COMPONENT_OVER_CS = {
    "D2Q9": math.sqrt(3.0),                       # D1Q3 product, nodes +-1 at c_s = 1/sqrt 3
    "D3Q27": math.sqrt(3.0),
    "D2Q19": 3.8358342053914734,                  # App. C, last row
    "D2Q25": math.sqrt(5.0 + math.sqrt(10.0)),    # outer root of He_5
    "D3Q13": math.sqrt((5.0 + math.sqrt(5.0)) / 2.0),  # r of Table tab:d3q13
    "D3Q21": ((1.0 + math.sqrt(5.0)) / 2.0) / math.sqrt(3.0 / 5.0),  # phi / c_s of Table tab:d3q21
    "D3V27": 3.142130383387586,                   # App. D, last row
    "D3Q45": 3.5256070994177073,                  # App. E, largest component
}

PERIODIC, EXTRAPOLATE = 0, 1


@dataclass(frozen=True)
class Workload:
    """Everything needed to create a lattice and its initial state."""

    name: str
    set: str
    grid: tuple          # (nx, ny, nz), nz = 1 in 2D
    dx: float
    dt: float
    cs: float
    tau: float
    order: int
    stencil: int
    steps: int
    compressible: bool = False
    gamma: float = 1.4
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)
    storage: str = "f64"
    log_every: int = 50
    support: str = "uniform"  # node placement: "uniform", or "glc" (cells of `stencil` GLC points)

    @property
    def D(self):
        return DIM[self.set]

    @property
    def shape(self):
        nx, ny, nz = self.grid
        return (nz, ny, nx)

    @property
    def ncell(self):
        return int(np.prod(self.grid))

    def with_(self, **kw):
        return replace(self, **kw)


def relaxation_time(nu: float, cs: float, dt: float) -> float:
    """tau = nu / (c_s^2 dt) + 1/2 (Sec. 3)."""
    return nu / (cs * cs * dt) + 0.5


def courant_dt(dx: float, cs: float, sets, courant: float = 0.5) -> float:
    """Time step at which the fastest component of the given sets moves
    ``courant`` cells per step."""
    vmax = max(MAX_COMPONENT_OVER_CS[s] for s in sets) * cs
    return courant * dx / vmax


def glc_nodes(n: int, p: int, dx: float):
    """Coordinates of the n nodes of a periodic axis divided into n / p cells
    of p + 1 Gauss-Lobatto-Chebyshev support points (the paper's cell-wise
    support, Sec. 3); neighbouring cells share their end points, and a cell
    is p dx wide, so the mean spacing is dx.  Node j = c p + k lies at
    (c + (1 - cos(pi k / p)) / 2) p dx."""
    if n % p:
        raise ValueError("%d nodes do not make whole cells of %d intervals" % (n, p))
    j = np.arange(n)
    c, k = j // p, j % p
    return (c + 0.5 * (1.0 - np.cos(np.pi * k / p))) * p * dx


def _axis(n, dx, glc_p=None):
    if glc_p:
        return glc_nodes(n, glc_p, dx)
    return np.arange(n, dtype=np.float64) * dx


def _grid_coords(shape, dx, glc_p=None):
    """Node coordinates (Z, Y, X) of a [nz][ny][nx] grid: uniform spacing dx,
    or Gauss-Lobatto-Chebyshev cells of glc_p intervals along every axis
    with more than one node."""
    nz, ny, nx = shape
    z = _axis(nz, dx, glc_p if nz > 1 else None)
    y = _axis(ny, dx, glc_p)
    x = _axis(nx, dx, glc_p)
    return np.meshgrid(z, y, x, indexing="ij")


def _coords(wl):
    return _grid_coords(wl.shape, wl.dx, wl.stencil - 1 if wl.support == "glc" else None)


# ---------------------------------------------------------------------------
# Workload 1: 2D Taylor-Green vortex, D2Q9, lattice units
# ---------------------------------------------------------------------------

def tgv2d_workload(n: int = 64, steps: int = 1000, Re: float = 100.0, storage: str = "f64",
                   set_: str = "D2Q9", stencil: int = 3) -> Workload:
    """D2Q9 in lattice units (dx = 1, c_s^2 = 1/3), dt = 0.5 so that every
    moving population shifts by 0.5 e_i; u0 = 0.05 c_s; the Reynolds number uses
    the box length L = n, so nu = u0 n / Re."""
    cs = 1.0 / math.sqrt(3.0)
    dt = 0.5
    u0 = 0.05 * cs
    nu = u0 * n / Re
    return Workload("tgv2d", set_, (n, n, 1), 1.0, dt, cs, relaxation_time(nu, cs, dt), 2, stencil, steps,
                    storage=storage)


def tgv2d_fields(wl: Workload, noise: float = 1e-6, seed: int = 0):
    """u = u0 (sin kx cos ky, -cos kx sin ky), k = 2 pi / n, and the matching
    pressure p' = (rho0 u0^2 / 4)(cos 2kx + cos 2ky) as rho = 1 + p'/c_s^2; each
    velocity component carries U(-noise, noise) from ``default_rng(seed)``."""
    nx, ny, _ = wl.grid
    u0 = 0.05 * wl.cs
    k = 2.0 * math.pi / (nx * wl.dx)
    _, Y, X = _coords(wl)
    ux = u0 * np.sin(k * X) * np.cos(k * Y)
    uy = -u0 * np.cos(k * X) * np.sin(k * Y)
    rho = 1.0 + (u0 * u0 / (4.0 * wl.cs * wl.cs)) * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    rng = np.random.default_rng(seed)
    u = np.stack([ux, uy])
    if noise:
        u = u + rng.uniform(-noise, noise, size=u.shape)
    return rho, u, None


def tgv2d_decay(wl: Workload, t: float) -> float:
    """Amplitude ratio exp(-2 nu k^2 t) of the 2D Taylor-Green velocity."""
    nu = (wl.tau - 0.5) * wl.cs ** 2 * wl.dt
    k = 2.0 * math.pi / (wl.grid[0] * wl.dx)
    return math.exp(-2.0 * nu * k * k * t)


# ---------------------------------------------------------------------------
# Workload 2 (and 5): weakly compressible 3D Taylor-Green vortex
# ---------------------------------------------------------------------------

TGV3D_SETS = ("D3Q13", "D3Q21", "D3V27", "D3Q27")


def tgv3d_workload(set_: str, n: int = 128, steps: int = 2000, Ma: float = 0.1, Re: float = 1600.0,
                   storage: str = "f32", stencil: int = 4, courant_sets=TGV3D_SETS,
                   order: int | None = None, support: str = "uniform") -> Workload:
    """Domain [0, 2 pi)^3 with n^3 nodes, u0 = 1, L = 1, c_s = 1/Ma, nu = 1/Re
    (Sec. 4.2); one time step for all sets in ``courant_sets`` at Courant 0.5
    (of the mean node spacing); N = 2, except N = 3 for D3V27 (Sec. 4.2).
    support="glc": the paper's own discretization, n/p cells of p + 1
    Gauss-Lobatto-Chebyshev points per axis with p = stencil - 1 (the paper's
    128^3 points are 32^3 cells with p = 4, Sec. 4.2)."""
    dx = 2.0 * math.pi / n
    cs = 1.0 / Ma
    dt = courant_dt(dx, cs, courant_sets)
    nu = 1.0 / Re
    if order is None:
        order = 3 if set_ == "D3V27" else 2
    return Workload("tgv3d", set_, (n, n, n), dx, dt, cs, relaxation_time(nu, cs, dt), order, stencil, steps,
                    storage=storage, support=support)


def tgv3d_pressure(X, Y, Z):
    """p' = (1/16)(cos 2x + cos 2y)(cos 2z + 2) for rho0 = u0 = 1 (Sec. 4.2; the
    printed 'cos(2z+2)' is read as cos 2z + 2, the form that solves the
    pressure Poisson equation of the given velocity)."""
    return (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0


def tgv3d_fields(wl: Workload, sigma: float = 0.0, seed: int = 1):
    """u = (sin x cos y cos z, -cos x sin y cos z, 0), rho = 1 + p'/c_s^2, plus an
    optional N(0, sigma^2) perturbation per component from ``default_rng(seed)``."""
    Z, Y, X = _coords(wl)
    u = np.stack([np.sin(X) * np.cos(Y) * np.cos(Z), -np.cos(X) * np.sin(Y) * np.cos(Z), np.zeros_like(X)])
    rho = 1.0 + tgv3d_pressure(X, Y, Z) / (wl.cs * wl.cs)
    if sigma:
        u = u + np.random.default_rng(seed).normal(0.0, sigma, size=u.shape)
    return rho, u, None


def adjoint_workload(n: int = 64, steps: int = 200, storage: str = "f32", Re: float = 1600.0) -> Workload:
    """D3Q27 Taylor-Green vortex for gradient checks: Ma 0.1, n = 4, N = 2,
    Courant 0.5 for D3Q27 alone."""
    return tgv3d_workload("D3Q27", n=n, steps=steps, Re=Re, storage=storage, courant_sets=("D3Q27",))


def fd_directions(shape_u, count: int = 16, seed: int = 2):
    """``count`` Gaussian direction fields with unit RMS, from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        v = rng.normal(size=shape_u)
        out.append(v / math.sqrt(np.mean(v * v)))
    return out


# ---------------------------------------------------------------------------
# Workload 4: compressible 3D Taylor-Green vortex (CTIC)
# ---------------------------------------------------------------------------

# Time steps of the paper's D3Q45 runs of the compressible Taylor-Green vortex
# (Table tab:timestepsizes, Re 400), by Mach number.
CTGV_PAPER_DT = {0.5: 0.0165, 1.0: 0.0329, 1.5: 0.0178, 2.0: 0.0119}


def ctgv_workload(n: int = 256, Ma: float = 0.5, Re: float = 1600.0, steps: int = 1000,
                  storage: str = "f32", set_: str = "D3Q45", stencil: int = 4, gamma: float = 1.4,
                  courant: float = 0.5, dt: float | None = None) -> Workload:
    """Domain [0, 2 pi)^3, u0 = 1, L = 1, rho0 = 1; the sound speed at theta = 1
    is c_s sqrt(gamma) = 1/Ma (Sec. 3: c_s* = c_s sqrt(theta gamma)); mu = 1/Re;
    N = 4 (Table tab:setup-full3Dvortex); tau quoted at rho theta = 1.  The
    time step is the one at the given Courant number of the fastest component,
    unless ``dt`` is given (e.g. ``CTGV_PAPER_DT[Ma]``)."""
    dx = 2.0 * math.pi / n
    cs = 1.0 / (Ma * math.sqrt(gamma))
    if dt is None:
        dt = courant_dt(dx, cs, (set_,), courant)
    return Workload("ctgv", set_, (n, n, n), dx, dt, cs, relaxation_time(1.0 / Re, cs, dt), 4, stencil, steps,
                    compressible=True, gamma=gamma, storage=storage)


def ctgv_fields(wl: Workload):
    """Constant-temperature initial condition (Sec. 4.3 with C = 1):
    rho = 1 + (1/16)(cos 2x + cos 2y)(cos 2z + 2), theta = 1, velocity of the
    Taylor-Green vortex."""
    Z, Y, X = _coords(wl)
    u = np.stack([np.sin(X) * np.cos(Y) * np.cos(Z), -np.cos(X) * np.sin(Y) * np.cos(Z), np.zeros_like(X)])
    rho = 1.0 + tgv3d_pressure(X, Y, Z)
    return rho, u, np.ones_like(rho)


# ---------------------------------------------------------------------------
# Workload 3: 2D shock-vortex interaction
# ---------------------------------------------------------------------------

def rankine_hugoniot(M1: float, gamma: float):
    """Normal-shock ratios rho2/rho1, P2/P1, T2/T1 and the downstream Mach number."""
    g = gamma
    r = (g + 1.0) * M1 * M1 / ((g - 1.0) * M1 * M1 + 2.0)
    p = 1.0 + 2.0 * g / (g + 1.0) * (M1 * M1 - 1.0)
    T = p / r
    M2 = math.sqrt((1.0 + 0.5 * (g - 1.0) * M1 * M1) / (g * M1 * M1 - 0.5 * (g - 1.0)))
    return r, p, T, M2


def svi_workload(set_: str = "D2Q19", n: int = 512, steps: int = 4000, storage: str = "f64",
                 Re: float = 800.0, Ma_a: float = 1.2, gamma: float = 1.4, stencil: int = 5) -> Workload:
    """Lattice units dx = 1, c_s = 1, upstream rho = theta = 1; R = n / 20
    (the paper's 60R x 24R box shrunk to a square 20R); dt = 0.002 R / c*_inf
    (Sec. 4.1); Re = c*_inf R / nu_inf; periodic in y, extrapolation in x;
    N = 4 and n = 5 (p = 4) per Table tab:setup-2Dvortex."""
    cs = 1.0
    R = n / 20.0
    c_star = cs * math.sqrt(gamma)
    dt = 0.002 * R / c_star
    nu = c_star * R / Re
    return Workload("svi", set_, (n, n, 1), 1.0, dt, cs, relaxation_time(nu, cs, dt), 4, stencil, steps,
                    compressible=True, gamma=gamma, bc=(EXTRAPOLATE, PERIODIC, PERIODIC), storage=storage)


def svi_fields(wl: Workload, Ma_v: float = 0.25, Ma_a: float = 1.2):
    """Steady Mach-``Ma_a`` shock at x = L/2 (Rankine-Hugoniot states, flow in
    +x) and an isentropic vortex of radius R = L/20 centred 2R upstream at
    (0.4 L, 0.5 L) (Sec. 4.1):
      u_theta = c* Ma_v r exp((1 - r^2)/2),
      P/P_inf = (1 - (gamma-1)/2 Ma_v^2 exp(1 - r^2))^(gamma/(gamma-1)),
      rho/rho_inf = (...)^(1/(gamma-1)),     r in units of R,
    reading Ma_v as Ma_v^2 in P and rho (the form in radial balance
    dP/dr = rho u_theta^2 / r).  Returns rho, u, theta with P = rho theta."""
    g = wl.gamma
    nx, ny, _ = wl.grid
    L = nx * wl.dx
    R = L / 20.0
    c_star = wl.cs * math.sqrt(g)
    ua = Ma_a * c_star
    r2, p2, T2, _ = rankine_hugoniot(Ma_a, g)
    _, Y, X = _grid_coords((1, ny, nx), wl.dx)
    down = X >= 0.5 * L
    rho = np.where(down, r2, 1.0)
    P = np.where(down, p2, 1.0)
    ux = np.where(down, ua / r2, ua)
    uy = np.zeros_like(X)
    # vortex upstream of the shock
    xc, yc = 0.4 * L, 0.5 * L
    dxv, dyv = (X - xc) / R, (Y - yc) / R
    rr2 = dxv * dxv + dyv * dyv
    rr = np.sqrt(rr2)
    ut = c_star * Ma_v * rr * np.exp(0.5 * (1.0 - rr2))
    with np.errstate(invalid="ignore", divide="ignore"):
        sin_t = np.where(rr > 0, dyv / np.where(rr > 0, rr, 1.0), 0.0)
        cos_t = np.where(rr > 0, dxv / np.where(rr > 0, rr, 1.0), 0.0)
    base = 1.0 - 0.5 * (g - 1.0) * Ma_v * Ma_v * np.exp(1.0 - rr2)
    up = ~down
    ux = np.where(up, ux - ut * sin_t, ux)
    uy = np.where(up, uy + ut * cos_t, uy)
    rho = np.where(up, base ** (1.0 / (g - 1.0)), rho)
    P = np.where(up, base ** (g / (g - 1.0)), P)
    theta = P / rho
    return rho, np.stack([ux, uy]), theta


# ---------------------------------------------------------------------------
# Small random states for parity tests
# ---------------------------------------------------------------------------

def random_fields(D: int, shape, seed: int, u_amp: float, rho_amp: float = 0.05, theta_amp: float = 0.0):
    """Smooth-free random fields: rho = 1 + U(-rho_amp, rho_amp),
    u = U(-u_amp, u_amp) per component, theta = 1 + U(-theta_amp, theta_amp)."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-rho_amp, rho_amp, size=shape)
    u = rng.uniform(-u_amp, u_amp, size=(D,) + tuple(shape))
    theta = None if theta_amp == 0.0 else 1.0 + rng.uniform(-theta_amp, theta_amp, size=shape)
    return rho, u, theta


def random_populations(nvals: int, shape, seed: int, base=None, amp: float = 0.1):
    """Random population-like arrays [nvals][shape] = base_i (1 + U(-amp, amp))."""
    rng = np.random.default_rng(seed)
    x = 1.0 + rng.uniform(-amp, amp, size=(nvals,) + tuple(shape))
    if base is not None:
        x = x * np.asarray(base).reshape((nvals,) + (1,) * len(shape))
    return x
