"""Adjoint kernels on the GPU.

* Transposition: <S v, w> = <v, S^T w> between the streaming and
  transposed-streaming kernels (FP64).
* Every adjoint kernel against the oracle's independent construction
  (complex-step Jacobians, scatter transpose): collision adjoint, fused
  reverse step, loss gradient, initial-equilibrium adjoint (FP64, 1e-12).
* The checkpointed rollout gradient against the oracle's gradient on a 16^3
  copy of the workload (FP64).
* The differentiation workload (D3Q27, 64^3, 200 steps, checkpoints every 20,
  loss = final kinetic energy, TGV plus N(0, 1e-3^2) perturbation): directional
  derivatives against central finite differences on 16 random directions,
  FP64, within 1e-6; the FP32 gradient within 5e-5 of the FP64 one.
"""
import numpy as np
import pytest
import torch

import lbm_inputs as W
from gpu_helpers import init_both, note, pair, rel_err, to_dev
from paper_2101_03982_amd import Lattice, kinetic_energy_after

pytestmark = pytest.mark.gpu


def dev_state(lat, a):
    return to_dev(a, lat.dtype).reshape(lat.pop_shape).contiguous()


@pytest.mark.parametrize("name,nx", [("D3Q27", 66), ("D3Q21", 66), ("D2Q19", 70), ("D3Q27", 67)])
def test_stream_transpose_dot_product(orc, name, nx):
    """An odd nx launches the single-load x variant of the 3D kernels."""
    grid = (nx, 9, 7) if W.DIM[name] == 3 else (nx, 21, 1)
    lat, cfg = pair(orc, name, grid, 0.6, 2, 4, "f64", dt=0.4)
    rng = np.random.default_rng(0)
    v = dev_state(lat, rng.normal(size=cfg.pop_shape()))
    w = dev_state(lat, rng.normal(size=cfg.pop_shape()))
    Sv, STw = lat.new_state(), lat.new_state()
    lat.stream_only(v, Sv)
    lat.adjoint_stream(w, STw)
    lhs = float(torch.sum(Sv * w))
    rhs = float(torch.sum(v * STw))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    # and both against the oracle
    assert rel_err(Sv.cpu().numpy(), orc.stream(cfg, v.cpu().numpy())) < 1e-13
    assert rel_err(STw.cpu().numpy(), orc.stream_transpose(cfg, w.cpu().numpy())) < 1e-13


@pytest.mark.parametrize("name,order,nx", [("D3Q27", 2, 66), ("D3V27", 2, 66), ("D2Q9", 2, 70), ("D3Q45", 2, 66),
                                           ("D3Q27", 2, 67)])
def test_adjoint_kernels_vs_oracle(orc, name, order, nx):
    """nx = 67: the single-load x variant of the adjoint kernels."""
    grid = (nx, 9, 7) if W.DIM[name] == 3 else (nx, 21, 1)
    cs = 0.6
    dt = 0.4 / (W.MAX_COMPONENT_OVER_CS[name] * cs)
    lat, cfg = pair(orc, name, grid, 0.57, order, 4, "f64", dt=dt, cs=cs)
    rho, u, _ = W.random_fields(cfg.D, cfg.shape, 1, 0.1 * cs)
    f0 = init_both(lat, orc, cfg, rho, u)
    fd = lat.state().clone()
    rng = np.random.default_rng(2)
    lam = rng.normal(size=cfg.pop_shape())
    nu_in = rng.normal(size=cfg.pop_shape())
    out = lat.new_state()
    # collision adjoint
    lat.adjoint_collide(fd, dev_state(lat, lam), out)
    ref = orc.adjoint_collide(cfg, orc.stream(cfg, f0), lam)
    assert rel_err(out.cpu().numpy(), ref) < 1e-12
    # fused reverse step
    lat.adjoint_step(fd, dev_state(lat, nu_in), out)
    ref = orc.adjoint_collide(cfg, orc.stream(cfg, f0), orc.stream_transpose(cfg, nu_in))
    assert rel_err(out.cpu().numpy(), ref) < 1e-12
    # loss gradient
    lat.ke_adjoint(fd, out)
    _, g = orc.ke_and_grad(cfg, f0)
    assert rel_err(out.cpu().numpy(), g) < 1e-12
    # initial equilibrium adjoint
    gu = torch.empty((cfg.D,) + cfg.shape, dtype=torch.float64, device="cuda:0")
    lat.init_equilibrium_adjoint(to_dev(rho, torch.float64), to_dev(u, torch.float64), dev_state(lat, lam), gu)
    assert rel_err(gu.cpu().numpy(), orc.init_transpose(cfg, rho, u, lam)) < 1e-12


@pytest.mark.parametrize("steps,every", [(20, 6), (200, 20)])
def test_rollout_gradient_vs_oracle(orc, steps, every):
    """The 16^3 copy of the differentiation workload: the full 200 steps with
    checkpoints every 20 (the workload's own), and a short run whose
    checkpoint interval does not divide the step count."""
    wl = W.adjoint_workload(n=16, storage="f64")
    lat, cfg = pair(orc, wl.set, wl.grid, wl.tau, wl.order, wl.stencil, "f64", wl.dx, wl.dt, wl.cs)
    rho, u, _ = W.tgv3d_fields(wl, sigma=1e-3, seed=1)
    u0 = to_dev(u, torch.float64).requires_grad_(True)
    K = kinetic_energy_after(u0, to_dev(rho, torch.float64), lat, steps, every=every)
    K.backward()
    loss, g = orc.ke_gradient_u0(cfg, rho, u, steps)
    assert abs(float(K.detach()) / loss - 1) < 1e-12
    assert rel_err(u0.grad.cpu().numpy(), g) < 1e-10


def _fd_check(storage, n=64, steps=200, ndir=16, h=1e-5):
    wl = W.adjoint_workload(n=n, steps=steps, storage=storage)
    lat = Lattice(wl.set, wl.grid, wl.tau, wl.order, stencil=wl.stencil, storage=storage, dx=wl.dx, dt=wl.dt,
                  cs=wl.cs, device="cuda:0")
    dt_ = lat.dtype
    rho_np, u_np, _ = W.tgv3d_fields(wl, sigma=1e-3, seed=1)
    rho = to_dev(rho_np, dt_)
    u0 = to_dev(u_np, dt_).requires_grad_(True)
    K = kinetic_energy_after(u0, rho, lat, steps, every=20)
    K.backward()
    grad = u0.grad.detach().double()
    dirs = W.fd_directions(u_np.shape, count=ndir, seed=2)
    out = []
    for v in dirs:
        vd = to_dev(v, dt_)
        kp = float(kinetic_energy_after(u0.detach() + h * vd, rho, lat, steps, every=steps))
        km = float(kinetic_energy_after(u0.detach() - h * vd, rho, lat, steps, every=steps))
        out.append(((kp - km) / (2 * h), float(torch.sum(grad * vd.double()))))
    return grad, out


def test_gradient_vs_finite_differences_fp64():
    _, pairs = _fd_check("f64")
    for fdv, adj in pairs:
        assert abs(adj - fdv) <= 1e-6 * abs(fdv), (adj, fdv)


def test_fp32_gradient_close_to_fp64():
    g64, _ = _fd_check("f64", ndir=0)
    g32, _ = _fd_check("f32", ndir=0)
    err = float(torch.linalg.norm(g32 - g64) / torch.linalg.norm(g64))
    worst = float(torch.max(torch.abs(g32 - g64)) / torch.max(torch.abs(g64)))
    note("adjoint_fp32_vs_fp64", rel_l2=err, max_rel=worst)
    # FP32 deviation storage rounds each step's populations to ~3e-8 of their
    # scale; over 200 forward and 200 reverse steps that is ~1e-5 (measured
    # 1.1e-5 rel. L2, 1.3e-5 worst element against the largest)
    assert err < 5e-5, err
    assert worst < 5e-5, worst
