"""Pins of the oracle's semi-Lagrangian streaming.

Sec. 3 (eq. sl_streaming) interpolates every population at its departure point
x - xi_i dt.  What fixes the result independently of the oracle's code:

* On-lattice shifts (xi_i dt / dx integer) make streaming a plain shift of the
  array, the "numpy.roll" of Sec. 5 -- bit for bit.
* A Lagrange interpolant through n nodes reproduces polynomials of degree
  <= n - 1; with extrapolating boundaries the interior of a polynomial field
  therefore streams to the polynomial evaluated at the departure point.
* A periodic Fourier mode exp(i k j) maps to G exp(i k j), where G is the value
  at the departure point of the polynomial through the mode's samples on the
  stencil nodes -- computed here with numpy's polynomial fit.
* Periodic streaming conserves each population's sum (the weights sum to 1).
* The worked example of the three-point stencil at shift 1/2 (tests/golden).
* Transpose: <S v, w> = <v, S^T w> between the gather (stream) and the
  scatter (stream_transpose), which are separate code.
"""
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=", 1)
                rows[k.strip()] = [float(x) for x in v.split()]
    return rows


@pytest.mark.parametrize("name,grid", [("D2Q9", (7, 5, 1)), ("D3Q27", (5, 4, 3))])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_on_lattice_is_a_roll(orc, name, grid, n):
    t = orc.table(name)
    cfg = orc.Config(name, grid, tau=1.0, stencil=n, dx=1.0, dt=1.0, cs=t["cs"])
    rng = np.random.default_rng(0)
    f = rng.uniform(0.5, 1.5, size=cfg.pop_shape())
    out = orc.stream(cfg, f)
    for i in range(cfg.Q):
        e = t["xi"][i].astype(int)
        # f_i(x) <- f_i(x - e): roll by +e along each axis (array axes z, y, x)
        shifts = tuple(int(e[a]) for a in reversed(range(cfg.D)))
        axes = tuple(range(3 - cfg.D, 3))
        exp = np.roll(f[i], shifts, axis=axes)
        assert np.array_equal(out[i], exp), (name, n, i)


@pytest.mark.parametrize("name", ["D2Q19", "D3Q21", "D3Q45"])
@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_polynomial_exactness(orc, name, n):
    """Interior nodes stream a degree-(n-1) polynomial exactly (extrapolating bc)."""
    t = orc.table(name)
    D = t["D"]
    grid = (19, 18, 17) if D == 3 else (19, 17, 1)
    dt = 0.37  # shifts of up to ~1.3 cells, fractional
    cfg = orc.Config(name, grid, tau=1.0, stencil=n, dx=1.0, dt=dt, bc=(1, 1, 1))
    shape = cfg.shape
    Z, Y, X = np.meshgrid(*[np.arange(s, dtype=float) for s in shape], indexing="ij")
    coeff = np.random.default_rng(n).uniform(-1, 1, size=(n, n, n))

    def poly(x, y, z):
        out = 0.0
        for a in range(n):
            for b in range(n):
                for c in range(n if D == 3 else 1):
                    out = out + coeff[a, b, c] * (x / 10) ** a * (y / 10) ** b * (z / 10) ** c
        return out

    p0 = poly(X, Y, Z)
    f = np.broadcast_to(p0, (cfg.Q,) + shape).copy()
    out = orc.stream(cfg, f)
    xi = t["xi"]
    reach = int(math.ceil(np.max(np.abs(xi)) * dt)) + n // 2 + 1
    for i in range(cfg.Q):
        s = xi[i] * dt
        exp = poly(X - s[0], Y - s[1], Z - (s[2] if D == 3 else 0.0))
        sl = tuple(slice(reach, -reach) for _ in range(3 - (3 - D))) if D == 3 else (slice(None),) + tuple(
            slice(reach, -reach) for _ in range(2))
        err = np.max(np.abs(out[i][sl] - exp[sl]))
        assert err <= 1e-12 * max(1.0, np.max(np.abs(exp))), (name, n, i, err)


def _nodes_for(s, n):
    """Stencil nodes relative to the arrival node: the n nodes around d = -s
    (even n), or centred on the node nearest d with ties to the arrival side
    (odd n)."""
    d = -s
    if n % 2 == 0:
        first = math.floor(d) - n // 2 + 1
    else:
        fl = math.floor(d)
        fr = d - fl
        c = fl if fr < 0.5 else fl + 1 if fr > 0.5 else (fl if abs(fl) <= abs(fl + 1) else fl + 1)
        first = c - (n - 1) // 2
    return np.arange(first, first + n)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
@pytest.mark.parametrize("s", [0.5, -0.5, 0.3, -1.7, 2.25])
def test_fourier_mode(orc, n, s):
    """exp(i k j) -> G exp(i k j) with G from numpy's polynomial interpolation."""
    N = 24
    cs = orc.table("D2Q9")["cs"]
    # population 3 of D2Q9 is xi = (+1, 0): shift s = dt
    cfg = orc.Config("D2Q9", (N, 3, 1), tau=1.0, stencil=n, dx=1.0, dt=s, cs=cs)
    xi = orc.table("D2Q9")["xi"]
    i = int(np.where((xi[:, 0] == 1) & (xi[:, 1] == 0))[0][0])
    jj = np.arange(N)
    for kk in (1, 3, 7):
        k = 2 * math.pi * kk / N
        f = np.ones(cfg.pop_shape())
        phase = 0.4
        f[i] = np.cos(k * jj + phase)[None, None, :]
        out = orc.stream(cfg, f)[i, 0, 1]
        nodes = _nodes_for(s, n)
        c = np.polynomial.polynomial.polyfit(nodes.astype(float), np.exp(1j * k * nodes), n - 1)
        G = np.polynomial.polynomial.polyval(-s, c)
        exp = np.real(G * np.exp(1j * (k * jj + phase)))
        assert np.max(np.abs(out - exp)) <= 1e-12, (n, s, kk)


@pytest.mark.parametrize("name", ["D2Q25", "D3Q13", "D3V27"])
@pytest.mark.parametrize("n", [3, 4])
def test_periodic_streaming_conserves_each_population(orc, name, n):
    D = orc.table(name)["D"]
    grid = (9, 8, 7) if D == 3 else (11, 9, 1)
    cfg = orc.Config(name, grid, tau=1.0, stencil=n, dx=0.5, dt=0.31)
    f = np.random.default_rng(1).uniform(0, 1, size=cfg.pop_shape())
    out = orc.stream(cfg, f)
    axes = tuple(range(1, 4))
    assert np.allclose(out.sum(axis=axes), f.sum(axis=axes), rtol=1e-13, atol=0)


def test_three_point_stencil_at_half_shift(orc):
    """Worked example (tests/golden/stencil_half_shift.txt): nodes {j-1, j, j+1},
    weights 3/8, 3/4, -1/8 for a shift of +1/2 cell."""
    g = load_golden("stencil_half_shift.txt")
    cs = orc.table("D2Q9")["cs"]
    N = 8
    cfg = orc.Config("D2Q9", (N, 3, 1), tau=1.0, stencil=3, dx=1.0, dt=0.5, cs=cs)
    xi = orc.table("D2Q9")["xi"]
    i = int(np.where((xi[:, 0] == 1) & (xi[:, 1] == 0))[0][0])
    f = np.zeros(cfg.pop_shape())
    f[i, 0, 1, 4] = 1.0  # delta at node 4
    out = orc.stream(cfg, f)[i, 0, 1]
    # f~(j) = sum_k L_k f(j + o_k): the delta at 4 is seen by j = 4 - o_k
    w = g["weights_shift_plus_half"]
    offs = [int(v) for v in g["offsets_shift_plus_half"]]
    exp = np.zeros(N)
    for o, wk in zip(offs, w):
        exp[4 - o] = wk
    assert np.array_equal(out, exp)


@pytest.mark.parametrize("name", ["D2Q19", "D3Q21"])
@pytest.mark.parametrize("bc", [0, 1])
def test_transpose_dot_product(orc, name, bc):
    D = orc.table(name)["D"]
    grid = (9, 7, 6) if D == 3 else (10, 9, 1)
    cfg = orc.Config(name, grid, tau=1.0, stencil=4, dx=1.0, dt=0.45, bc=(bc, 0, bc))
    rng = np.random.default_rng(5)
    v = rng.normal(size=cfg.pop_shape())
    w = rng.normal(size=cfg.pop_shape())
    lhs = np.sum(orc.stream(cfg, v) * w)
    rhs = np.sum(v * orc.stream_transpose(cfg, w))
    assert lhs == pytest.approx(rhs, rel=1e-13)
