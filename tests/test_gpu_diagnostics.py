"""Enstrophy diagnostic (Sec. 4.2) on the GPU.

* Parity: the HIP kernel against the oracle (``oracle/diagnostics.py``) on
  the same velocity fields, FP64 and FP32 inputs, 2D and 3D, orders 2-8, grids
  with ragged tiles and grids shorter than the stencil (periodic wrap): within
  1e-12 (both sides take FP64 arithmetic on the same values).
* The state's own velocity (``enstrophy()`` without a field) equals the
  oracle's enstrophy of the velocity that ``moments()`` returns.
* Errors: a clamped axis is unsupported, an odd order is rejected.
* The weakly compressible Taylor-Green run: the kinetic energy lost against
  the physical dissipation nu int E dt; the difference is the scheme's
  numerical dissipation, 15-21 % on the 128^3 workload, under 1 % at 256^3.
"""
import numpy as np
import pytest
import torch

import lbm_inputs as W
from gpu_helpers import to_dev
from oracle import diagnostics as G
from paper_2101_03982_amd import Lattice
from paper_2101_03982_amd._lib import LBM_EINVAL, LBM_EUNSUPPORTED, LbmError

pytestmark = pytest.mark.gpu


def velocity(D, shape, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    Z, Y, X = np.meshgrid(np.arange(nz) / nz, np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")
    u = np.stack([np.sin(2 * np.pi * (X + 2 * Y + (c + 1) * Z) + c) for c in range(D)])
    return u + 0.3 * rng.normal(size=u.shape)


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("name,grid", [("D3Q27", (70, 13, 9)), ("D3Q27", (5, 4, 4)), ("D2Q9", (70, 21, 1)),
                                       ("D2Q9", (3, 7, 1))])
@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_enstrophy_parity(storage, name, grid, order):
    dx = 0.37
    lat = Lattice(name, grid, 0.8, 2, stencil=4, storage=storage, dx=dx, dt=0.1, cs=1.0, device="cuda:0")
    u = velocity(lat.D, lat.shape, seed=order)
    ud = to_dev(u, lat.dtype)
    got = lat.enstrophy(ud, order=order)
    ref = G.enstrophy(ud.double().cpu().numpy(), dx, order)
    assert abs(got / ref - 1) <= 1e-12, (got, ref)


def test_enstrophy_of_the_state(orc):
    wl = W.tgv3d_workload("D3Q27", n=32)
    lat = Lattice("D3Q27", wl.grid, wl.tau, wl.order, stencil=wl.stencil, storage="f32", dx=wl.dx, dt=wl.dt,
                  cs=wl.cs, device="cuda:0")
    rho, u, _ = W.tgv3d_fields(wl)
    lat.init_equilibrium(to_dev(rho, torch.float32), to_dev(u, torch.float32))
    lat.step(20)
    _, uu, _, _ = lat.moments()
    got = lat.enstrophy()
    ref = G.enstrophy(uu.double().cpu().numpy(), wl.dx, 8)
    assert abs(got / ref - 1) <= 1e-12


def test_enstrophy_errors():
    lat = Lattice("D2Q9", (70, 21), 0.8, 2, stencil=4, storage="f64", dx=1.0, dt=0.5,
                  boundary=("extrapolate", "periodic", "periodic"), device="cuda:0")
    u = torch.zeros((2,) + lat.shape, dtype=torch.float64, device="cuda:0")
    with pytest.raises(LbmError) as e:
        lat.enstrophy(u)
    assert e.value.code == LBM_EUNSUPPORTED
    lat = Lattice("D2Q9", (70, 21), 0.8, 2, stencil=4, storage="f64", dx=1.0, dt=0.5, device="cuda:0")
    with pytest.raises(LbmError) as e:
        lat.enstrophy(u, order=5)
    assert e.value.code == LBM_EINVAL


def dissipation_excess(name, n, t_end=1.5625, logs=40):
    """Weakly compressible Taylor-Green run (Sec. 4.2) at n^3, FP32: the
    kinetic energy lost, K(0) - K(t), over the physical dissipation
    nu int_0^t E dt (trapezoidal in the log), minus one, at t_end and at its
    half; the acoustic exchange with the compressive energy averages out of
    the integrated balance."""
    wl = W.tgv3d_workload(name, n=n)
    lat = Lattice(name, wl.grid, wl.tau, wl.order, stencil=wl.stencil, storage="f32", dx=wl.dx, dt=wl.dt,
                  cs=wl.cs, device="cuda:0")
    rho, u, _ = W.tgv3d_fields(wl)
    lat.init_equilibrium(to_dev(rho, torch.float32), to_dev(u, torch.float32))
    steps = int(round(t_end / wl.dt))
    every = steps // logs
    ke, ens, t = [], [], []
    done = 0
    while True:
        _, uu, _, d = lat.moments()
        ke.append(d.ke)
        ens.append(lat.enstrophy(uu))
        t.append(done * wl.dt)
        if done >= steps:
            break
        k = min(every, steps - done)
        lat.step(k)
        done += k
    lat.close()
    del lat
    torch.cuda.empty_cache()
    ke, ens, t = np.array(ke), np.array(ens), np.array(t)
    nu = 1.0 / 1600.0
    phys = nu * np.concatenate([[0.0], np.cumsum(0.5 * (ens[1:] + ens[:-1]) * np.diff(t))])
    excess = (ke[0] - ke[1:]) / phys[1:] - 1
    return ens[0], excess[len(excess) // 2 - 1], excess[-1]


@pytest.mark.parametrize("name", W.TGV3D_SETS)
def test_tgv_dissipation_balance(name):
    """Sec. 4.2: nu E is the physical dissipation rate, and -dK/dt beyond it is
    numerical dissipation.  At 256^3 (resolved) the kinetic energy lost up to
    t = 0.78 and t = 1.56 equals nu int E dt within 1 %; on the 128^3 workload
    the interpolation adds 5-40 % (measured 15-21 %), which refinement
    removes.  E(0) is the closed form 3/4 of the initial field."""
    e0, mid128, end128 = dissipation_excess(name, 128)
    _, mid256, end256 = dissipation_excess(name, 256)
    print(name, "excess 128^3: %.4f %.4f  256^3: %.4f %.4f" % (mid128, end128, mid256, end256))
    assert e0 == pytest.approx(0.75, rel=2e-3)
    assert abs(mid256) < 0.01 and abs(end256) < 0.01
    assert 0.05 < mid128 < 0.4 and 0.05 < end128 < 0.4
