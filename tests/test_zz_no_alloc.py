"""lbm_moments_noalloc (the allocation-free variant of lbm_moments, for
callers that cannot allocate) through the C ABI against lbm_moments: per-cell
rho, u, theta and the global diagnostics agree bit for bit, on two calls in a
row, the second on a smaller lattice (fewer reduction blocks, so block sums
left in the shared static array by the first call must not be read)."""
import ctypes

import numpy as np
import pytest
import torch

import lbm_inputs as W
from paper_2101_03982_amd import Lattice, _lib

pytestmark = pytest.mark.gpu


def _both(lat):
    """(fields, diag) from lbm_moments and from lbm_moments_noalloc."""
    out = []
    for name in ("lbm_moments", "lbm_moments_noalloc"):
        rho = torch.full(lat.shape, float("nan"), dtype=lat.dtype, device=lat.device)
        u = torch.full((lat.D,) + lat.shape, float("nan"), dtype=lat.dtype, device=lat.device)
        th = torch.full(lat.shape, float("nan"), dtype=lat.dtype, device=lat.device)
        d = _lib.Diag()
        lat._stream()
        rc = getattr(_lib.lib(), name)(lat._ctx, None, ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                       ctypes.c_void_p(th.data_ptr()), ctypes.byref(d))
        assert rc == 0, (name, _lib.lib().lbm_last_error())
        diag = (d.mass, tuple(d.momentum), d.ke, d.energy, d.min_rho, d.min_theta, d.nonfinite)
        out.append(([x.cpu().numpy() for x in (rho, u, th)], diag))
    return out


def _lattice(name, grid, comp, storage, seed):
    D = W.DIM[name]
    cs = 0.6
    dt = 0.4 / (W.MAX_COMPONENT_OVER_CS[name] * cs)
    lat = Lattice(name, grid, 0.7, 4 if comp else 2, stencil=4, storage=storage, dt=dt, cs=cs, compressible=comp,
                  device="cuda:0")
    rho, u, theta = W.random_fields(D, lat.shape, seed, u_amp=0.1 * cs, rho_amp=0.03,
                                    theta_amp=0.05 if comp else 0.0)
    dev = lambda a: None if a is None else torch.from_numpy(a).to("cuda:0", lat.dtype)  # noqa: E731
    lat.init_equilibrium(dev(rho), dev(u), dev(theta))
    lat.step(2)
    return lat


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_noalloc_moments_match_twice_then_smaller(storage):
    # first call: 96 x 64 x 48 cells = 1152 blocks' worth -> all 1024 blocks;
    # second call: 40 x 20 x 10 cells -> 32 blocks (stale sums beyond them)
    cases = [("D3Q45", (96, 64, 48), True), ("D3Q27", (40, 20, 10), False)]
    for k, (name, grid, comp) in enumerate(cases):
        lat = _lattice(name, grid, comp, storage, seed=30 + k)
        (f_ref, d_ref), (f_new, d_new) = _both(lat)
        assert d_new == d_ref, (name, d_new, d_ref)
        for a, b in zip(f_new, f_ref):
            assert np.array_equal(a, b, equal_nan=False), name
        assert d_ref[6] == 0 and d_ref[4] > 0
        lat.close()
