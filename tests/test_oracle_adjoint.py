"""Pins of the oracle's adjoint pieces (gradient checks; not part of the paper).

The oracle differentiates its own forward code by complex steps and applies
the transpose of streaming as a scatter.  These tests pin both against central
finite differences of the plain FP64 forward map, which shares nothing with
the reverse accumulation except the forward functions themselves.
"""
import numpy as np
import pytest

import lbm_inputs as W


def fd(fun, x, v, h):
    return (fun(x + h * v) - fun(x - h * v)) / (2 * h)


@pytest.mark.parametrize("name,N,comp", [("D2Q9", 2, False), ("D3Q27", 2, False), ("D3V27", 3, False),
                                         ("D3Q45", 4, True)])
def test_collision_jacobian_vs_fd(orc, name, N, comp):
    cfg = orc.Config(name, (1, 1, 1), tau=0.62, order=N, stencil=1, compressible=comp)
    cs = orc.table(name)["cs"]
    base = orc.feq(cfg, 1.01, np.array([0.1, -0.05, 0.07])[:cfg.D] * cs, 1.05 if comp else 1.0)
    rng = np.random.default_rng(0)
    f = base * (1 + rng.uniform(-0.05, 0.05, size=base.shape))
    J = orc.collide_jacobian(cfg, f)
    for _ in range(4):
        v = rng.normal(size=f.shape) * np.abs(base)
        num = fd(lambda x: orc.collide_one(cfg, x), f, v, 1e-6)
        assert np.allclose(J @ v, num, rtol=0, atol=1e-8 * np.max(np.abs(num)))


def test_ke_gradient_vs_fd(orc):
    cfg = orc.Config("D3Q13", (4, 3, 3), tau=0.6, order=2, stencil=3, dx=1.0, dt=0.3)
    rho, u, _ = W.random_fields(3, cfg.shape, 1, 0.1)
    f = orc.init(cfg, rho, u)
    ke, g = orc.ke_and_grad(cfg, f)
    v = np.random.default_rng(2).normal(size=f.shape) * 1e-2
    num = fd(lambda x: orc.ke_and_grad(cfg, x, want_grad=False)[0], f, v, 1e-5)
    assert np.sum(g * v) == pytest.approx(num, rel=1e-8)


def test_init_transpose_vs_fd(orc):
    cfg = orc.Config("D2Q19", (5, 4, 1), tau=0.6, order=4, stencil=3, dx=1.0, dt=0.3)
    rho, u, _ = W.random_fields(2, cfg.shape, 3, 0.2)
    rng = np.random.default_rng(4)
    lam = rng.normal(size=cfg.pop_shape())
    g = orc.init_transpose(cfg, rho, u, lam)
    v = rng.normal(size=u.shape)
    num = fd(lambda x: np.sum(lam * orc.init(cfg, rho, x)), u, v, 1e-6)
    assert np.sum(g * v) == pytest.approx(num, rel=1e-8)


@pytest.mark.parametrize("name,grid,bc", [("D2Q9", (6, 5, 1), (0, 0, 0)), ("D3Q27", (4, 4, 3), (0, 0, 0)),
                                          ("D2Q25", (6, 5, 1), (1, 0, 0))])
def test_full_gradient_vs_fd(orc, name, grid, bc):
    """d k(f_T) / d u0 by reverse accumulation vs central differences of the
    forward map, FP64, along random directions."""
    t = orc.table(name)
    cfg = orc.Config(name, grid, tau=0.58, order=2, stencil=4, dx=1.0, dt=0.4 / (t["cs"] / t["cs"]),
                     cs=t["cs"], bc=bc)
    rho, u, _ = W.random_fields(cfg.D, cfg.shape, 5, 0.1 * t["cs"])
    steps = 3
    loss, g = orc.ke_gradient_u0(cfg, rho, u, steps)

    def forward(uu):
        f = orc.run(cfg, orc.init(cfg, rho, uu), steps)
        return orc.ke_and_grad(cfg, f, want_grad=False)[0]

    assert loss == pytest.approx(forward(u), rel=1e-14)
    rng = np.random.default_rng(6)
    for _ in range(3):
        v = rng.normal(size=u.shape)
        num = fd(forward, u, v, 1e-6)
        assert np.sum(g * v) == pytest.approx(num, rel=2e-8)
