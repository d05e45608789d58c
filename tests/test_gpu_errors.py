"""Failure handling on the GPU: divergence detection, argument checks of the
binding, and the stream contract (no test makes a kernel fault or hang)."""
import numpy as np
import pytest
import torch

import lbm_inputs as W
from paper_2101_03982_amd import Lattice
from paper_2101_03982_amd._lib import LBM_EDIVERGED, LbmError

pytestmark = pytest.mark.gpu


def small(storage="f32", compressible=False, name="D3Q27", order=2):
    return Lattice(name, (66, 9, 7), 0.6, order, stencil=4, storage=storage, dt=0.3, cs=0.6,
                   compressible=compressible, device="cuda:0")


def test_negative_density_is_reported():
    lat = small()
    rho = torch.ones(lat.shape, device="cuda:0")
    rho[3, 4, 5] = -0.5
    u = torch.zeros((3,) + lat.shape, device="cuda:0")
    lat.init_equilibrium(rho, u)
    with pytest.raises(LbmError) as e:
        lat.moments()
    assert e.value.code == LBM_EDIVERGED


def test_nan_is_reported_and_counted():
    lat = small("f64")
    rho = torch.ones(lat.shape, device="cuda:0", dtype=torch.float64)
    u = torch.zeros((3,) + lat.shape, device="cuda:0", dtype=torch.float64)
    lat.init_equilibrium(rho, u)
    lat.state()[5, 1, 2, 3] = float("nan")
    lat.step(1)  # spreads to the stencil's neighbours
    with pytest.raises(LbmError) as e:
        lat.moments()
    assert e.value.code == LBM_EDIVERGED


def test_negative_temperature_is_reported():
    lat = small("f64", compressible=True, name="D3Q45", order=4)
    rho = torch.ones(lat.shape, device="cuda:0", dtype=torch.float64)
    u = torch.zeros((3,) + lat.shape, device="cuda:0", dtype=torch.float64)
    th = torch.ones(lat.shape, device="cuda:0", dtype=torch.float64)
    th[0, 0, 0] = -0.2
    lat.init_equilibrium(rho, u, th)
    with pytest.raises(LbmError) as e:
        lat.moments()
    assert e.value.code == LBM_EDIVERGED


def test_binding_checks_dtype_and_shape():
    lat = small("f32")
    with pytest.raises(ValueError):
        lat.init_equilibrium(torch.ones(lat.shape, device="cuda:0", dtype=torch.float64),
                             torch.zeros((3,) + lat.shape, device="cuda:0"))
    with pytest.raises(ValueError):
        lat.init_equilibrium(torch.ones((5, 5), device="cuda:0"), torch.zeros((3,) + lat.shape, device="cuda:0"))


def test_work_follows_the_current_stream():
    lat = small("f64")
    rho = torch.ones(lat.shape, device="cuda:0", dtype=torch.float64)
    u = 0.01 * torch.ones((3,) + lat.shape, device="cuda:0", dtype=torch.float64)
    lat.init_equilibrium(rho, u)
    ref = lat.state().clone()
    lat2 = small("f64")
    lat2.init_equilibrium(rho, u)
    lat.step(3)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        lat2.step(3)
        out = lat2.state().clone()
    torch.cuda.synchronize()
    assert torch.equal(out, lat.state())
    assert not torch.equal(ref, lat.state())


def test_adjoint_unsupported_for_deviation_storage():
    lat = Lattice("D3Q27", (66, 9, 7), 0.6, 2, stencil=4, storage="bf16", dt=0.3, cs=0.6, device="cuda:0")
    a, b = lat.new_state(), lat.new_state()
    with pytest.raises(LbmError):
        lat.adjoint_stream(a, b)
