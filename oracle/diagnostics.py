"""Flow diagnostics of Sec. 4.2 in plain FP64 numpy: kinetic energy, enstrophy
and the velocity-gradient norms that check it.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares nothing
with the GPU library.

Velocities are float64 arrays ``[D][nz][ny][nx]`` (x fastest) on a uniform
periodic grid of spacing ``dx``.  Sec. 4.2 defines the kinetic energy as the
domain mean of |u|^2/2 and the enstrophy as the domain mean of |curl u|^2; on
the periodic uniform grid the domain mean is the mean over the nodes.  The
derivatives are central differences of order 2m whose coefficients are found
here from their defining Taylor conditions (exact for odd powers up to
2m - 1), not from a closed form.
"""
from __future__ import annotations

import numpy as np

# axis of each coordinate in a component array [nz][ny][nx]
_AXIS = {0: 2, 1: 1, 2: 0}


def central_difference_weights(m: int) -> np.ndarray:
    """a_1..a_m with f'(x) ~ sum_j a_j (f(x + j h) - f(x - j h)) / h exact for
    polynomials of degree <= 2m: the odd powers x^(2k+1), k < m, give
    sum_j 2 a_j j^(2k+1) = [k == 0] (even powers cancel by symmetry)."""
    j = np.arange(1, m + 1, dtype=np.float64)
    A = np.array([2.0 * j ** (2 * k + 1) for k in range(m)])
    b = np.zeros(m)
    b[0] = 1.0
    return np.linalg.solve(A, b)


def derivative(f: np.ndarray, coord: int, dx: float, order: int) -> np.ndarray:
    """d f / d x_coord of a periodic field [nz][ny][nx], central differences of
    the given even order."""
    a = central_difference_weights(order // 2)
    ax = _AXIS[coord]
    out = np.zeros_like(f)
    for j, aj in enumerate(a, start=1):
        # np.roll(f, -j)[i] = f[i + j]
        out += aj * (np.roll(f, -j, axis=ax) - np.roll(f, j, axis=ax))
    return out / dx


def curl(u: np.ndarray, dx: float, order: int = 8) -> np.ndarray:
    """Vorticity curl u: three components in 3D, the z component in 2D."""
    D = u.shape[0]
    d = lambda comp, coord: derivative(u[comp], coord, dx, order)  # noqa: E731
    if D == 2:
        return np.stack([d(1, 0) - d(0, 1)])
    return np.stack([d(2, 1) - d(1, 2), d(0, 2) - d(2, 0), d(1, 0) - d(0, 1)])


def kinetic_energy(u: np.ndarray) -> float:
    """<|u|^2 / 2> over the nodes (Sec. 4.2)."""
    return float(np.mean(0.5 * np.sum(u * u, axis=0)))


def enstrophy(u: np.ndarray, dx: float, order: int = 8) -> float:
    """<|curl u|^2> over the nodes (Sec. 4.2)."""
    w = curl(u, dx, order)
    return float(np.mean(np.sum(w * w, axis=0)))


def gradient_norms(u: np.ndarray, dx: float, order: int = 8):
    """<sum_ab (d_a u_b)^2> and <(div u)^2> with the same derivatives: on a
    periodic grid <|curl u|^2> = <|grad u|^2> - <(div u)^2> for any commuting
    skew-symmetric difference operators, a check of the curl's components."""
    D = u.shape[0]
    g = [[derivative(u[b], a, dx, order) for b in range(D)] for a in range(D)]
    grad2 = float(np.mean(sum(g[a][b] ** 2 for a in range(D) for b in range(D))))
    div2 = float(np.mean(sum(g[a][a] for a in range(D)) ** 2))
    return grad2, div2


def spectral_enstrophy(u: np.ndarray, dx: float) -> float:
    """<|curl u|^2> from the exact derivatives of the field's trigonometric
    interpolant (Parseval: the mean of |i k x u_hat|^2 over the modes)."""
    D = u.shape[0]
    shape = u.shape[1:]
    ks = [2 * np.pi * np.fft.fftfreq(n, d=dx) for n in shape]  # per axis [z, y, x]
    K = np.meshgrid(*ks, indexing="ij")
    k = {0: K[2], 1: K[1], 2: K[0]}
    uh = [np.fft.fftn(u[c]) for c in range(D)]
    if D == 2:
        wh = [1j * (k[0] * uh[1] - k[1] * uh[0])]
    else:
        wh = [1j * (k[1] * uh[2] - k[2] * uh[1]), 1j * (k[2] * uh[0] - k[0] * uh[2]),
              1j * (k[0] * uh[1] - k[1] * uh[0])]
    n = np.prod(shape)
    return float(sum(np.sum(np.abs(w) ** 2) for w in wh) / n ** 2)
