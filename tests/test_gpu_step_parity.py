"""GPU time step vs the FP64 CPU oracle, element by element.

Grids span several 64-wide x tiles, several y/z tiles and a ragged tail on
every axis; populations start at the equilibrium of seeded random fields with
the velocity amplitude of the paper's weakly compressible runs.  The bar:
FP64 storage within 1e-12 of the oracle relative to the largest population;
FP32 within 3e-6 of each population's own scale (its largest deviation from
its reference value w_i over the cells: a few FP32 roundings per tap and per
collision term of the deviations it stores); BF16 and FP16 storage within
three units of their format's roundoff of each population's scale."""
import numpy as np
import pytest
import torch

import lbm_inputs as W
from gpu_helpers import gpu_populations, init_both, note, pair, pop_err, reference_values, rel_err, to_dev
from paper_2101_03982_amd import Lattice

pytestmark = pytest.mark.gpu

SETS = ["D2Q9", "D2Q19", "D2Q25", "D3Q13", "D3Q21", "D3Q27", "D3V27", "D3Q45"]
TOL = {"f64": 1e-12, "f32": 3e-6}


def check(lat, got, ref, storage, case, factor=1.0):
    """FP64: relative to the largest population; FP32: per population."""
    if storage == "f64":
        err = rel_err(got, ref)
    else:
        err = pop_err(lat, got, ref)
    note(case, err=err)
    assert err <= TOL[storage] * factor, (case, err)


def grid_for(D):
    return (70, 13, 7) if D == 3 else (70, 21, 1)


def problem(orc, name, storage, n, order=2, dt_cells=0.45, steps=3, seed=0, grid=None):
    D = W.DIM[name]
    grid = grid or grid_for(D)
    cs = 0.6
    # shifts of up to dt_cells cells along the fastest component
    dt = dt_cells / (W.MAX_COMPONENT_OVER_CS[name] * cs)
    lat, cfg = pair(orc, name, grid, tau=0.57, order=order, n=n, storage=storage, dx=1.0, dt=dt, cs=cs)
    rho, u, _ = W.random_fields(D, cfg.shape, seed, u_amp=0.1 * cs, rho_amp=0.02)
    f0 = init_both(lat, orc, cfg, rho, u)
    lat.step(steps)
    ref = orc.run(cfg, f0, steps)
    return lat, gpu_populations(lat), ref


@pytest.mark.parametrize("name", SETS)
@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_step_parity_all_sets(orc, name, storage):
    lat, got, ref = problem(orc, name, storage, n=4)
    check(lat, got, ref, storage, "all_sets_%s_%s" % (name, storage))


# unit roundoff of the 16-bit storage formats
ULP = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}


@pytest.mark.parametrize("name", ["D3Q13", "D3Q21", "D3V27", "D3Q27"])
@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_reduced_precision_weak_sets_one_step(orc, name, storage):
    """BF16/FP16 deviation storage for the weakly compressible 3D sets at
    their workload order (N = 2; N = 3 for D3V27), n = 4, on a ragged grid:
    one step from the equilibrium, each stored value within three units of
    the format's roundoff of its population's largest deviation from w_i,
    against the FP64 oracle (the rounding of the initial state, interpolated,
    plus the rounding of the result; 2^-23 more for FP16's subnormals)."""
    order = 3 if name == "D3V27" else 2
    lat, got, ref = problem(orc, name, storage, n=4, order=order, steps=1)
    check16(lat, got, ref, storage, "weak16_%s_%s" % (name, storage))


def check16(lat, got, ref, storage, case):
    """One step of 16-bit storage: each value within three units of the
    format's roundoff of its population's largest deviation from w_i."""
    r = reference_values(lat).reshape((-1, 1, 1, 1))
    scale = np.max(np.abs(ref - r), axis=(1, 2, 3), keepdims=True)
    tol = 3 * ULP[storage] * scale + 2.0 ** -23
    note(case, err=float(np.max(np.abs(got - ref) / tol)))
    assert np.all(np.abs(got - ref) <= tol), float(np.max(np.abs(got - ref) / tol))


@pytest.mark.parametrize("name", ["D2Q9", "D2Q19", "D3Q13", "D3Q27", "D3Q45"])
@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_step_parity_stencil_lengths(orc, name, n):
    lat, got, ref = problem(orc, name, "f64", n=n)
    check(lat, got, ref, "f64", "stencil_%s_%d" % (name, n))


@pytest.mark.parametrize("name,order", [("D3V27", 3), ("D2Q25", 4), ("D2Q19", 4), ("D3Q45", 4)])
def test_step_parity_higher_orders(orc, name, order):
    lat, got, ref = problem(orc, name, "f64", n=4, order=order)
    check(lat, got, ref, "f64", "order_%s_%d" % (name, order))


@pytest.mark.parametrize("name", ["D2Q19", "D3Q21", "D3Q45"])
def test_large_courant_number(orc, name):
    """Shifts of several cells (the paper's large time steps, Sec. 4.3)."""
    grid = (70, 13, 12) if W.DIM[name] == 3 else (70, 21, 1)
    lat, got, ref = problem(orc, name, "f64", n=4, dt_cells=3.7, steps=2, grid=grid)
    check(lat, got, ref, "f64", "courant_%s" % name)


def test_zero_steps_is_a_no_op(orc):
    lat, cfg = pair(orc, "D3Q13", (66, 5, 5), tau=0.6, n=4, storage="f64", dt=0.2)
    rho, u, _ = W.random_fields(3, cfg.shape, 1, 0.05)
    init_both(lat, orc, cfg, rho, u)
    before = lat.state().clone()
    lat.step(0)
    assert np.array_equal(before.cpu().numpy(), lat.state().cpu().numpy())


@pytest.mark.parametrize("name,storage,comp", [("D3Q27", "f64", False), ("D3Q21", "f32", False),
                                               ("D3Q45", "f32", True)])
def test_minimal_grid(orc, name, storage, comp):
    """The smallest periodic grid the stencil allows: one tile, every axis a
    tail (also for the eight-wave blocks of D3Q21 and the FP32 f + g model)."""
    cs = 0.6
    dt = 0.3 / (W.MAX_COMPONENT_OVER_CS[name] * cs)
    lat, cfg = pair(orc, name, (6, 6, 6), tau=0.7, order=4 if comp else 2, n=4, storage=storage, dt=dt, cs=cs,
                    compressible=comp)
    rho, u, theta = W.random_fields(3, cfg.shape, 4, 0.1 * cs, theta_amp=0.05 if comp else 0.0)
    f0 = init_both(lat, orc, cfg, rho, u, theta)
    lat.step(2)
    got, ref = gpu_populations(lat), orc.run(cfg, f0, 2)
    check(lat, got, ref, storage, "minimal_%s_%s" % (name, storage), factor=3 if comp else 1)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("grid,bc", [((67, 9, 6), (0, 0, 0)), ((70, 9, 6), (1, 0, 0))])
def test_x_pair_load_fallbacks(orc, storage, grid, bc):
    """3D populations load x in pairs of adjacent nodes when x is periodic
    with nx even; an odd nx (a pair would straddle the wrap) and a clamped x
    boundary (pairs not adjacent) launch the single-load kernels."""
    name = "D3Q27"
    cs = 0.6
    dt = 0.45 / (W.MAX_COMPONENT_OVER_CS[name] * cs)
    lat, cfg = pair(orc, name, grid, tau=0.57, order=2, n=4, storage=storage, dx=1.0, dt=dt, cs=cs, bc=bc)
    rho, u, _ = W.random_fields(3, cfg.shape, 5, u_amp=0.1 * cs, rho_amp=0.02)
    f0 = init_both(lat, orc, cfg, rho, u)
    steps = 1 if storage in ULP else 2
    lat.step(steps)
    ref = orc.run(cfg, f0, steps)
    case = "xpair_%s_%s_%d" % (storage, "".join(map(str, bc)), grid[0])
    if storage in ULP:
        check16(lat, gpu_populations(lat), ref, storage, case)
    else:
        check(lat, gpu_populations(lat), ref, storage, case)


@pytest.mark.parametrize("name,storage,bc,n,comp", [
    ("D3Q27", "f64", (0, 1, 1), 4, False),
    ("D3Q27", "f32", (1, 1, 1), 4, False),
    ("D3Q21", "f64", (0, 0, 1), 3, False),
    ("D3Q45", "f32", (0, 1, 0), 4, True),
    ("D2Q19", "f64", (0, 1, 0), 5, True),
    ("D2Q9", "f32", (1, 1, 0), 3, False),
])
def test_extrapolating_axes(orc, name, storage, bc, n, comp):
    """Zeroth-order extrapolation (node indices clamped to the edge) along y
    and z as well as x: two steps against the oracle on a ragged grid, with
    shifts of up to 1.3 cells so that stencils reach past both edges."""
    D = W.DIM[name]
    grid = (70, 13, 7) if D == 3 else (70, 21, 1)
    cs = 0.6
    dt = 1.3 / (W.MAX_COMPONENT_OVER_CS[name] * cs)
    order = 4 if comp else 2
    lat, cfg = pair(orc, name, grid, tau=0.7, order=order, n=n, storage=storage, dx=1.0, dt=dt, cs=cs,
                    compressible=comp, bc=bc)
    rho, u, theta = W.random_fields(D, cfg.shape, 13, u_amp=0.1 * cs, rho_amp=0.02,
                                    theta_amp=0.03 if comp else 0.0)
    f0 = init_both(lat, orc, cfg, rho, u, theta)
    lat.step(2)
    ref = orc.run(cfg, f0, 2)
    check(lat, gpu_populations(lat), ref, storage, "extrap_%s_%s_%s" % (name, storage, "".join(map(str, bc))),
          factor=3 if comp else 1)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16", "f16"])
def test_unaligned_buffers_match_aligned(orc, storage):
    """Buffers starting one element off an even address launch the
    single-load kernels; the step is the same to the last bit."""
    import torch

    name = "D3Q21"
    cs = 0.6
    dt = 0.45 / (W.MAX_COMPONENT_OVER_CS[name] * cs)
    lat, cfg = pair(orc, name, (66, 9, 6), tau=0.57, order=2, n=4, storage=storage, dx=1.0, dt=dt, cs=cs)
    rho, u, _ = W.random_fields(3, cfg.shape, 6, u_amp=0.1 * cs, rho_amp=0.02)
    init_both(lat, orc, cfg, rho, u)
    f0 = lat.state().clone()
    out_a = lat.new_state()
    lat.step_into(f0, out_a)
    n = f0.numel()
    big_src = torch.zeros(n + 1, dtype=f0.dtype, device=f0.device)
    big_dst = torch.zeros(n + 1, dtype=f0.dtype, device=f0.device)
    src = big_src[1:].view(f0.shape)
    dst = big_dst[1:].view(f0.shape)
    src.copy_(f0)
    lat.step_into(src, dst)
    torch.cuda.synchronize()
    ints = {"f64": torch.int64, "f32": torch.int32}.get(storage, torch.int16)
    assert torch.equal(dst.view(ints), out_a.view(ints))


@pytest.mark.parametrize("storage,small", [("f32", (128, 128, 64)), ("f64", (128, 64, 64)),
                                           ("bf16", (128, 128, 128))])
def test_streamed_stores_match_cached_stores(storage, small):
    """When the two state buffers exceed the 256 MB last-level cache, the 3D
    n = 4 step stores its results with the non-temporal cache policy.  The
    values are the same bit for bit: a D3Q27 lattice holding two periodic
    copies (along z) of a smaller one whose two buffers fit (226 MB, cached
    stores; the doubled lattice 453 MB, streamed stores) steps to two copies
    of the smaller one's result, for FP32, FP64 and BF16 storage."""
    name = "D3Q27"
    cs = 0.6
    dt = 0.45 / (W.MAX_COMPONENT_OVER_CS[name] * cs)
    kw = dict(stencil=4, storage=storage, dx=1.0, dt=dt, cs=cs, device="cuda:0")
    nx, ny, nz = small
    lo = Lattice(name, small, 0.57, 2, **kw)
    hi = Lattice(name, (nx, ny, 2 * nz), 0.57, 2, **kw)
    rho, u, _ = W.random_fields(3, lo.shape, 21, u_amp=0.1 * cs, rho_amp=0.02)
    lo.init_equilibrium(to_dev(rho, lo.dtype), to_dev(u, lo.dtype))
    hi.init_equilibrium(to_dev(np.concatenate([rho, rho], axis=0), hi.dtype),
                        to_dev(np.concatenate([u, u], axis=1), hi.dtype))
    lo.step(3)
    hi.step(3)
    ints = {"f32": torch.int32, "f64": torch.int64, "bf16": torch.int16}[storage]
    a = lo.state().view(ints)
    b = hi.state().view(ints)
    assert torch.equal(b[:, :nz], a) and torch.equal(b[:, nz:], a)
