"""Throughput of the semi-Lagrangian lattice Boltzmann step on one MI355X.

Workload: the weakly compressible 3D Taylor-Green vortex on a 128^3 periodic
grid in FP32 with the four velocity sets of Sec. 4.2 (D3Q13, D3Q21, D3V27,
D3Q27), tricubic Lagrange streaming (n = 4) at Courant number 0.5, Ma 0.1,
Re 1600, N = 2 (N = 3 for D3V27); kinetic energy logged every 50 steps.  One
bench step advances all four lattices by one time step.  Inputs are the
analytic initial fields, resident in HBM before timing starts.

Prints one JSON line: MLUPS of the whole workload, per-set MLUPS and fraction
of HBM peak, the roofline of the dominant kernel (HIP-event timing of single
launches on the lattice's stream), and the FP64 CPU oracle timed on a bounded
sample of the same workload on this host's cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import contextlib
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
SETS = ("D3Q13", "D3Q21", "D3V27", "D3Q27")
KERNEL_SRC = os.path.join(ROOT, "paper_2101_03982_amd", "csrc", "lbm_kernels.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=128, help="grid points per axis")
    ap.add_argument("--log-every", type=int, default=None,
                    help="kinetic-energy log interval in steps (default: 50, or --steps if fewer, so that the "
                         "timed window always holds at least one log)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the FP64-error, adjoint-cost, dissipation, reduced-precision and high-Mach measurements")
    ap.add_argument("--precision-n", type=int, default=256)
    ap.add_argument("--precision-steps", type=int, default=1000)
    ap.add_argument("--sets", default=",".join(SETS))
    ap.add_argument("--streams", type=int, default=0,
                    help="streams the lattices step on (0: one per lattice, 1: all on the current stream)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--only", default=None,
                    help="run one leg alone and print its JSON (precision, svi, svi2048, adjoint, large_grid, glc, "
                         "prandtl); "
                         "with --precision-steps and --storages it is the profiling target of one kernel family")
    ap.add_argument("--storages", default="f64,f32,bf16,f16", help="storages of the precision leg")
    ap.add_argument("--machs", default="0.5,1.0", help="Mach numbers of the precision leg")
    a = ap.parse_args()
    if a.log_every is None:
        a.log_every = min(50, a.steps)
    return a


def kernel_sha():
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_for(set_name, n):
    """HBM bytes per launch from the committed PMC counters, if they were taken
    with the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha():
        return None
    e = t.get("kernels", {}).get("%s_%d" % (set_name, n))
    return None if e is None else e.get("bytes_per_launch")


def cpu_baseline(sets, n, steps=3):
    """The FP64 oracle, `steps` time steps of every set at the full grid size
    (a bounded sample of the workload: about 10-20 s on 16 host cores)."""
    import lbm_inputs as W
    from oracle import oracle as O

    O.build()
    t_total = 0.0
    cells = 0
    for s in sets:
        wl = W.tgv3d_workload(s, n=n)
        cfg = O.Config(wl.set, wl.grid, tau=wl.tau, order=wl.order, stencil=wl.stencil, dx=wl.dx, dt=wl.dt,
                       cs=wl.cs)
        rho, u, _ = W.tgv3d_fields(wl)
        f = O.init(cfg, rho, u)
        t0 = time.perf_counter()
        f = O.run(cfg, f, steps)
        t_total += time.perf_counter() - t0
        cells += wl.ncell * steps
        del f
    return {"value": cells / t_total / 1e6, "unit": "MLUPS", "cores": O.num_threads(), "kind": "oracle",
            "sample": "%d FP64 time steps of each of %s on the %d^3 grid (%.1f s)" % (steps, "/".join(sets), n,
                                                                                  t_total)}


def fp64_error(sets, n, steps, ke32):
    """KE of an FP64 run of the same workload after the same number of steps,
    and the FP32 run's relative deviation from it."""
    import torch

    import lbm_inputs as W
    from paper_2101_03982_amd import Lattice

    out = {}
    for s in sets:
        wl = W.tgv3d_workload(s, n=n)
        lat = Lattice(s, wl.grid, wl.tau, wl.order, stencil=wl.stencil, storage="f64", dx=wl.dx, dt=wl.dt,
                      cs=wl.cs, device="cuda:0")
        rho, u, _ = W.tgv3d_fields(wl)
        lat.init_equilibrium(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
        lat.step(steps)
        ke64 = lat.moments(fields=False)[3].ke
        out[s] = {"ke_fp64": ke64, "ke_fp32": ke32[s], "ke_rel_err": abs(ke32[s] / ke64 - 1)}
        lat.close()
        del lat
    return out


def adjoint_cost(n=64, steps=200, every=20):
    """Differentiation workload: D3Q27, FP32, loss = final kinetic energy,
    gradient w.r.t. the initial velocity with checkpoints every `every` steps.
    Times the forward (with checkpointing) and the backward (recompute +
    adjoint kernels) with CUDA events."""
    import torch

    import lbm_inputs as W
    from paper_2101_03982_amd import Lattice, kinetic_energy_after

    wl = W.adjoint_workload(n=n, steps=steps, storage="f32")
    lat = Lattice(wl.set, wl.grid, wl.tau, wl.order, stencil=wl.stencil, storage="f32", dx=wl.dx, dt=wl.dt,
                  cs=wl.cs, device="cuda:0")
    rho_np, u_np, _ = W.tgv3d_fields(wl, sigma=1e-3, seed=1)
    rho = torch.from_numpy(rho_np).to("cuda:0", torch.float32)
    times = []
    for rep in range(3):
        u0 = torch.from_numpy(u_np).to("cuda:0", torch.float32).requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        K = kinetic_energy_after(u0, rho, lat, steps, every=every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        K.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
    fwd, bwd = min(times, key=lambda t: t[0] + t[1])
    g32 = u0.grad.detach().double()
    # plain forward without checkpoints, for reference
    lat.init_equilibrium(rho, torch.from_numpy(u_np).to("cuda:0", torch.float32))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat.step(steps)
    torch.cuda.synchronize()
    plain = time.perf_counter() - t0
    lat.close()
    # the same gradient in FP64: the FP32 gradient's deviation from it
    wl64 = W.adjoint_workload(n=n, steps=steps, storage="f64")
    lat64 = Lattice(wl64.set, wl64.grid, wl64.tau, wl64.order, stencil=wl64.stencil, storage="f64", dx=wl64.dx,
                    dt=wl64.dt, cs=wl64.cs, device="cuda:0")
    u64 = torch.from_numpy(u_np).to("cuda:0", torch.float64).requires_grad_(True)
    kinetic_energy_after(u64, torch.from_numpy(rho_np).to("cuda:0", torch.float64), lat64, steps,
                         every=every).backward()
    g64 = u64.grad.detach()
    lat64.close()
    return {"workload": "D3Q27 %d^3 FP32, %d steps, checkpoints every %d, loss = final kinetic energy" % (
        n, steps, every), "forward_s": fwd, "backward_s": bwd, "plain_forward_s": plain,
        "adjoint_over_forward": bwd / fwd, "adjoint_over_plain_forward": bwd / plain,
        "fp32_grad_rel_l2_vs_fp64": float(torch.linalg.norm(g32 - g64) / torch.linalg.norm(g64)),
        "fp32_grad_max_rel_vs_fp64": float(torch.max(torch.abs(g32 - g64)) / torch.max(torch.abs(g64)))}


def dissipation(sets=SETS, n=128, t_end=1.5625, logs=40):
    """Sec. 4.2's split of the kinetic-energy decay of the weakly compressible
    Taylor-Green run into the physical dissipation nu E (E = <|curl u|^2>, the
    library's enstrophy kernel, eighth-order differences) and the rest, the
    scheme's numerical dissipation: (K(0) - K(t)) / (nu int_0^t E dt) - 1."""
    import numpy as np
    import torch

    import lbm_inputs as W
    from paper_2101_03982_amd import Lattice

    res = {}
    for s in sets:
        wl = W.tgv3d_workload(s, n=n)
        lat = Lattice(s, wl.grid, wl.tau, wl.order, stencil=wl.stencil, storage="f32", dx=wl.dx, dt=wl.dt,
                      cs=wl.cs, device="cuda:0")
        rho, u, _ = W.tgv3d_fields(wl)
        lat.init_equilibrium(torch.from_numpy(rho).to("cuda:0", torch.float32),
                             torch.from_numpy(u).to("cuda:0", torch.float32))
        steps = int(round(t_end / wl.dt))
        every = steps // logs
        ke, ens, t, ens_ms = [], [], [], []
        done = 0
        while True:
            _, uu, _, d = lat.moments()
            t0 = time.perf_counter()
            ens.append(lat.enstrophy(uu))
            ens_ms.append((time.perf_counter() - t0) * 1e3)
            ke.append(d.ke)
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
        phys = (1.0 / 1600.0) * np.concatenate([[0.0], np.cumsum(0.5 * (ens[1:] + ens[:-1]) * np.diff(t))])
        excess = (ke[0] - ke[1:]) / phys[1:] - 1
        res[s] = {"numerical_over_physical_t%.2f" % t[len(t) // 2]: round(float(excess[len(excess) // 2 - 1]), 4),
                  "numerical_over_physical_t%.2f" % t[-1]: round(float(excess[-1]), 4),
                  "enstrophy_t0": round(float(ens[0]), 6), "enstrophy_end": round(float(ens[-1]), 6),
                  "enstrophy_call_ms": round(float(np.median(ens_ms)), 3)}
    res["workload"] = "3D Taylor-Green vortex %d^3 FP32, Re 1600, to t = %g, enstrophy every %d steps" % (
        n, t_end, every)
    return res


def high_mach(n=256, t_end=10.0, machs=(0.5, 1.0, 1.5, 2.0), storage="f32", every=50):
    """Compressible TGV with D3Q45 at the paper's own time steps (Table
    tab:timestepsizes, Re 400) to t = t_end: time per step, whether the run
    stayed finite with rho > 0 and theta > 0, and its kinetic-energy decay."""
    import math

    import torch

    import lbm_inputs as W
    from paper_2101_03982_amd import Lattice

    res = {}
    for Ma in machs:
        wl = W.ctgv_workload(n=n, Ma=Ma, Re=400.0, dt=W.CTGV_PAPER_DT[Ma] * 256.0 / n)
        steps = int(math.ceil(t_end / wl.dt))
        lat = Lattice("D3Q45", wl.grid, wl.tau, 4, stencil=wl.stencil, storage=storage, dx=wl.dx, dt=wl.dt,
                      cs=wl.cs, compressible=True, gamma=wl.gamma, device="cuda:0")
        rho_np, u_np, th_np = W.ctgv_fields(wl)
        dt_ = lat.dtype
        lat.init_equilibrium(torch.from_numpy(rho_np).to("cuda:0", dt_), torch.from_numpy(u_np).to("cuda:0", dt_),
                             torch.from_numpy(th_np).to("cuda:0", dt_))
        d0 = lat.moments(fields=False)[3]
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        done, ms, ok, lo_rho, lo_th, d = 0, 0.0, True, d0.min_rho, d0.min_theta, d0
        while done < steps:
            k = min(every, steps - done)
            e0.record()
            lat.step(k)
            e1.record()
            try:
                d = lat.moments(fields=False)[3]
            except Exception as exc:  # noqa: BLE001 - reported in the JSON
                ok = "stopped at step %d: %s" % (done + k, str(exc)[:100])
                break
            ms += e0.elapsed_time(e1)
            done += k
            lo_rho, lo_th = min(lo_rho, d.min_rho), min(lo_th, d.min_theta)
        res["Ma%.1f" % Ma] = {
            "dt": wl.dt, "tau": round(wl.tau, 4), "steps": steps,
            "max_shift_cells": round(W.MAX_COMPONENT_OVER_CS["D3Q45"] * wl.cs * wl.dt / wl.dx, 3),
            "stable": ok, "t_reached": round(done * wl.dt, 3),
            "ms_per_step": round(ms / max(done, 1), 4), "ke_ratio": round(d.ke / d0.ke, 5),
            "min_rho": round(lo_rho, 4), "min_theta": round(lo_th, 4),
            "mass_drift": abs(d.mass / d0.mass - 1), "energy_drift": abs(d.energy / d0.energy - 1)}
        lat.close()
        del lat
        torch.cuda.empty_cache()
    res["workload"] = ("compressible TGV (CTIC) D3Q45 f+g, N = 4, n = 4, %d^3, Re 400, the paper's time steps, "
                       "%s, to t = %g" % (n, storage.upper(), t_end))
    return res


def precision_form(n=256, steps=1000, machs=(0.5, 1.0),
                   storages=("f64", "f32", "bf16", "bf16_sr", "f16", "f16_sr")):
    """Compressible TGV with D3Q45 (N = 4, n = 4): time per step and error
    after `steps` steps of the BF16/FP16 deviation storage (*_sr: stochastic
    rounding) and of FP32 against the FP64 run on the same GPU."""
    import numpy as np
    import torch

    import lbm_inputs as W
    from paper_2101_03982_amd import Lattice

    res = {}
    for Ma in machs:
        wl = W.ctgv_workload(n=n, Ma=Ma)
        rho_np, u_np, th_np = W.ctgv_fields(wl)
        ref = None
        entry = {}
        for st in storages:
            sto = st[:-3] if st.endswith("_sr") else st
            lat = Lattice("D3Q45", wl.grid, wl.tau, 4, stencil=wl.stencil, storage=sto, dx=wl.dx, dt=wl.dt,
                          cs=wl.cs, compressible=True, gamma=wl.gamma,
                          energy_f64=(sto in ("bf16", "f16") and Ma >= 1.0),
                          rounding="stochastic" if st.endswith("_sr") else "nearest", device="cuda:0")
            dt_ = lat.dtype
            lat.init_equilibrium(torch.from_numpy(rho_np).to("cuda:0", dt_), torch.from_numpy(u_np).to("cuda:0", dt_),
                                 torch.from_numpy(th_np).to("cuda:0", dt_))
            warm = min(5, steps - 1)
            lat.step(warm)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            lat.step(steps - warm)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / (steps - warm)
            try:
                r, u, th, d = lat.moments()
                fields = (r.double(), u.double(), th.double())
                ok = True
            except Exception as exc:  # noqa: BLE001 - reported in the JSON
                fields, d, ok = None, None, str(exc)
            bpc = 2 * 90 * {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[sto]
            gbs = bpc * wl.ncell / (ms * 1e-3) / 1e9
            e = {"ms_per_step": ms, "mlups": wl.ncell / (ms * 1e-3) / 1e6, "bytes_per_cell": bpc,
                 "achieved_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS, "ok": ok}
            if ok is True:
                e["ke"] = d.ke
                if st == "f64":
                    ref = fields
                elif ref is not None:
                    def rl2(a, b):
                        return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
                    e["rel_l2_rho"] = rl2(fields[0], ref[0])
                    e["rel_l2_u"] = rl2(fields[1], ref[1])
                    e["rel_l2_theta"] = rl2(fields[2], ref[2])
                    e["ke_rel_err"] = abs(d.ke / entry["f64"]["ke"] - 1)
            entry[st] = e
            lat.close()
            del lat
            torch.cuda.empty_cache()
        for st in ("bf16", "bf16_sr", "f16", "f16_sr"):
            if "f32" in entry and st in entry:
                entry["speedup_%s_over_f32" % st] = entry["f32"]["ms_per_step"] / entry[st]["ms_per_step"]
        res["Ma%.1f" % Ma] = entry
    res["workload"] = "compressible TGV (CTIC) D3Q45 f+g, N = 4, n = 4, %d^3, Re 1600, %d steps" % (n, steps)
    return res


def copy_reference(nbytes):
    """A plain device-to-device copy moving the same bytes as one launch of
    the dominant kernel (read + write): the bandwidth a streaming kernel can
    reach on this machine, beside the nominal peak."""
    import torch

    n = nbytes // 2 // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 50
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / reps * 1e3
    del x, y
    torch.cuda.empty_cache()
    return {"bytes": 2 * n * 4, "us": us, "GBs": 2 * n * 4 / (us * 1e-6) / 1e9}


def kernel_time(lat, reps=50):
    """Average single-launch time (ms) of lat.step(1) with HIP events on the
    lattice's stream."""
    import torch

    stream = torch.cuda.current_stream()
    lat.step(3)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in evs:
        e0.record(stream)
        lat.step(1)
        e1.record(stream)
    torch.cuda.synchronize()
    return sum(e0.elapsed_time(e1) for e0, e1 in evs) / reps


def large_grid(sets=("D3Q13", "D3Q27"), n=256):
    """The same kernels on a 256^3 grid, whose two buffers exceed the 256 MB
    Infinity Cache, so the bandwidth figure is HBM's."""
    import torch

    import lbm_inputs as W
    from paper_2101_03982_amd import Lattice

    out = {}
    for s in sets:
        wl = W.tgv3d_workload(s, n=n)
        lat = Lattice(s, wl.grid, wl.tau, wl.order, stencil=wl.stencil, storage="f32", dx=wl.dx, dt=wl.dt,
                      cs=wl.cs, device="cuda:0")
        rho, u, _ = W.tgv3d_fields(wl)
        lat.init_equilibrium(torch.from_numpy(rho).to("cuda:0", torch.float32),
                             torch.from_numpy(u).to("cuda:0", torch.float32))
        ms = kernel_time(lat)
        gbs = 2 * lat.Q * 4 * wl.ncell / (ms * 1e-3) / 1e9
        out[s] = {"kernel_ms": ms, "mlups": wl.ncell / (ms * 1e-3) / 1e6, "achieved_GBs": gbs,
                  "hbm_frac": gbs / HBM_PEAK_GBS}
        lat.close()
        del lat
        torch.cuda.empty_cache()
    out["workload"] = "3D Taylor-Green vortex %d^3 FP32, n = 4 (working set above the Infinity Cache)" % n
    return out


def on_lattice_ratio(n=128):
    """Context for the paper's cost statement (Sec. 5: semi-Lagrangian
    streaming costs about ten times on-lattice streaming): D3Q27 FP32 at n^3
    with integer shifts (streaming is a plain shift) against the tricubic
    off-lattice step of the Taylor-Green workload, single-launch times."""
    import math

    import torch

    import lbm_inputs as W
    from paper_2101_03982_amd import Lattice

    out = {}
    wl = W.tgv3d_workload("D3Q27", n=n)
    rho, u, _ = W.tgv3d_fields(wl)
    cases = {"on_lattice": dict(dx=1.0, dt=1.0, cs=1.0 / math.sqrt(3.0), tau=0.6),
             "semi_lagrangian": dict(dx=wl.dx, dt=wl.dt, cs=wl.cs, tau=wl.tau)}
    for name, c in cases.items():
        lat = Lattice("D3Q27", wl.grid, c["tau"], 2, stencil=4, storage="f32", dx=c["dx"], dt=c["dt"], cs=c["cs"],
                      device="cuda:0")
        lat.init_equilibrium(torch.from_numpy(rho).to("cuda:0", torch.float32),
                             torch.from_numpy(u * (c["cs"] / wl.cs)).to("cuda:0", torch.float32))
        out[name + "_ms"] = kernel_time(lat)
        lat.close()
        del lat
        torch.cuda.empty_cache()
    out["ratio"] = out["semi_lagrangian_ms"] / out["on_lattice_ms"]
    out["workload"] = "D3Q27 %d^3 FP32: integer shifts (1-node copy) vs n = 4 Lagrange streaming" % n
    return out


def glc_throughput(sets=("D3Q13", "D3Q21", "D3V27", "D3Q27"), n=128):
    """The paper's own streaming support on the Taylor-Green workload's grid:
    32^3 cells of p = 4 Gauss-Lobatto-Chebyshev points (128^3 nodes, Sec.
    4.2), FP32, single-launch time per set beside the uniform tricubic step."""
    import torch

    import lbm_inputs as W
    from paper_2101_03982_amd import Lattice

    out = {}
    for s in sets:
        wl = W.tgv3d_workload(s, n=n, stencil=5, support="glc")
        lat = Lattice(s, wl.grid, wl.tau, wl.order, stencil=5, storage="f32", dx=wl.dx, dt=wl.dt, cs=wl.cs,
                      support="glc", device="cuda:0")
        rho, u, _ = W.tgv3d_fields(wl)
        lat.init_equilibrium(torch.from_numpy(rho).to("cuda:0", torch.float32),
                             torch.from_numpy(u).to("cuda:0", torch.float32))
        ms = kernel_time(lat)
        gbs = 2 * lat.Q * 4 * wl.ncell / (ms * 1e-3) / 1e9
        out[s] = {"kernel_ms": ms, "mlups": wl.ncell / (ms * 1e-3) / 1e6, "achieved_GBs": gbs,
                  "hbm_frac": gbs / HBM_PEAK_GBS}
        lat.close()
        del lat
        torch.cuda.empty_cache()
    out["workload"] = ("3D Taylor-Green vortex %d^3 nodes = %d^3 cells of p = 4 Gauss-Lobatto-Chebyshev points, "
                       "FP32, cell-wise streaming" % (n, n // 4))
    return out


def prandtl_cost(Pr=0.75):
    """The quasi-equilibrium collision for Pr != 1 against plain BGK: single-
    launch time of the precision workload's FP32 and FP64 kernels (D3Q45 f+g
    256^3, Ma 1.0) and of the 2048^2 shock-vortex D2Q19 kernels, Pr = 0.75."""
    import torch

    import lbm_inputs as W
    from paper_2101_03982_amd import Lattice

    out = {}
    wl = W.ctgv_workload(n=256, Ma=1.0)
    rho, u, th = W.ctgv_fields(wl)
    for st in ("f64", "f32"):
        for pr in (1.0, Pr):
            lat = Lattice("D3Q45", wl.grid, wl.tau, 4, stencil=wl.stencil, storage=st, dx=wl.dx, dt=wl.dt, cs=wl.cs,
                          compressible=True, gamma=wl.gamma, prandtl=pr, device="cuda:0")
            dt_ = lat.dtype
            lat.init_equilibrium(torch.from_numpy(rho).to("cuda:0", dt_), torch.from_numpy(u).to("cuda:0", dt_),
                                 torch.from_numpy(th).to("cuda:0", dt_))
            out["D3Q45_256_%s_Pr%g_ms" % (st, pr)] = kernel_time(lat, reps=10)
            lat.close()
            del lat
            torch.cuda.empty_cache()
    sw = W.svi_workload("D2Q19", n=2048, storage="f32")
    r2, u2, t2 = W.svi_fields(sw)
    for st in ("f64", "f32"):
        for pr in (1.0, Pr):
            lat = Lattice("D2Q19", sw.grid, sw.tau, sw.order, stencil=sw.stencil, storage=st, dx=sw.dx, dt=sw.dt,
                          cs=sw.cs, compressible=True, gamma=sw.gamma, prandtl=pr,
                          boundary=("extrapolate", "periodic", "periodic"), device="cuda:0")
            dt_ = lat.dtype
            lat.init_equilibrium(torch.from_numpy(r2).to("cuda:0", dt_), torch.from_numpy(u2).to("cuda:0", dt_),
                                 torch.from_numpy(t2).to("cuda:0", dt_))
            out["D2Q19_2048_%s_Pr%g_ms" % (st, pr)] = kernel_time(lat)
            lat.close()
            del lat
            torch.cuda.empty_cache()
    out["workload"] = "quasi-equilibrium (Pr = %g) vs BGK: D3Q45 f+g 256^3 Ma 1.0; D2Q19 f+g 2048^2 shock-vortex" % Pr
    return out


def svi_throughput(n=512):
    """Shock-vortex workload (D2Q19 / D2Q25, f + g, N = 4, n = 5, extrapolating
    in x) at n^2 (512^2, the workload's size, whose two buffers fit in the
    256 MB Infinity Cache; 2048^2, 1.3-3.4 GB, for HBM's rate): single-launch
    time per set and storage."""
    import torch

    import lbm_inputs as W
    from paper_2101_03982_amd import Lattice

    out = {}
    for s in ("D2Q19", "D2Q25"):
        for st in ("f64", "f32"):
            wl = W.svi_workload(s, n=n, storage=st)
            lat = Lattice(s, wl.grid, wl.tau, wl.order, stencil=wl.stencil, storage=st, dx=wl.dx, dt=wl.dt,
                          cs=wl.cs, compressible=True, gamma=wl.gamma,
                          boundary=("extrapolate", "periodic", "periodic"), device="cuda:0")
            rho, u, th = W.svi_fields(wl)
            dt_ = lat.dtype
            lat.init_equilibrium(torch.from_numpy(rho).to("cuda:0", dt_), torch.from_numpy(u).to("cuda:0", dt_),
                                 torch.from_numpy(th).to("cuda:0", dt_))
            ms = kernel_time(lat)
            b = 8 if st == "f64" else 4
            gbs = 2 * 2 * lat.Q * b * wl.ncell / (ms * 1e-3) / 1e9
            out["%s_%s" % (s, st)] = {"kernel_ms": ms, "mlups": wl.ncell / (ms * 1e-3) / 1e6, "achieved_GBs": gbs,
                                      "hbm_frac": gbs / HBM_PEAK_GBS}
            lat.close()
            del lat
            torch.cuda.empty_cache()
    out["workload"] = "2D shock-vortex interaction %d^2, D2Q19/D2Q25 f+g, N = 4, n = 5" % n
    return out


def run_only(a):
    """One leg alone (profiling target)."""
    legs = {
        "precision": lambda: precision_form(a.precision_n, a.precision_steps,
                                            tuple(float(m) for m in a.machs.split(",")),
                                            tuple(a.storages.split(","))),
        "svi": lambda: svi_throughput(512),
        "svi2048": lambda: svi_throughput(2048),
        "adjoint": adjoint_cost,
        "large_grid": large_grid,
        "glc": glc_throughput,
        "prandtl": prandtl_cost,
    }
    if a.only not in legs:
        print("unknown leg %r (one of %s)" % (a.only, ", ".join(sorted(legs))), file=sys.stderr)
        sys.exit(2)
    if a.copy_probe:
        copy_probe()
    print(json.dumps({"leg": a.only, a.only: legs[a.only]()}), flush=True)


def copy_probe():
    """A plain 1 GiB device-to-device copy (1 GiB read, 1 GiB written): the
    known-size kernel that calibrates the HBM byte counters."""
    import torch

    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    torch.cuda.empty_cache()


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path (got --gpus %d)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch

    import lbm_inputs as W
    from paper_2101_03982_amd import Lattice

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if a.only:
        run_only(a)
        return
    dev = torch.device("cuda:0")
    sets = tuple(a.sets.split(","))
    if a.copy_probe:
        copy_probe()
    lats = []
    for s in sets:
        wl = W.tgv3d_workload(s, n=a.n)
        lat = Lattice(s, wl.grid, wl.tau, wl.order, stencil=wl.stencil, storage="f32", dx=wl.dx, dt=wl.dt,
                      cs=wl.cs, device=dev)
        rho, u, _ = W.tgv3d_fields(wl)
        lat.init_equilibrium(torch.from_numpy(rho).to(dev, torch.float32),
                             torch.from_numpy(u).to(dev, torch.float32))
        lats.append((s, wl, lat))
    torch.cuda.synchronize()

    ke_log = {s: [] for s in sets}
    # the lattices are independent: each steps on a stream of its own (default
    # priority) so that one kernel's last blocks overlap the next one's first
    nstreams = len(lats) if a.streams <= 0 else a.streams
    streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)] if nstreams > 1 else None

    def one_step(k):
        for i, (s, _, lat) in enumerate(lats):
            ctx = torch.cuda.stream(streams[i % nstreams]) if streams else contextlib.nullcontext()
            with ctx:
                lat.step(1)
                if a.log_every and (k + 1) % a.log_every == 0:
                    _, _, _, d = lat.moments(fields=False)
                    ke_log[s].append(d.ke)

    for k in range(a.warmup):
        one_step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        one_step(k)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # per-launch kernel time with HIP events on the lattices' stream
    stream = torch.cuda.current_stream(dev)
    per_set = {}
    reps = 50
    for s, wl, lat in lats:
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in evs:
            e0.record(stream)
            lat.step(1)
            e1.record(stream)
        torch.cuda.synchronize()
        ms = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
        avg_ms = sum(ms) / len(ms)
        # the diagnostics call (moments kernel, block-sum reduction, 72-byte copy
        # to the host; it waits for the stream), separately from the step
        mom = []
        for _ in range(10):
            m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            m0.record(stream)
            lat.moments(fields=False)
            m1.record(stream)
            torch.cuda.synchronize()
            mom.append(m0.elapsed_time(m1))
        bpc = 2 * lat.Q * 4  # one FP32 read and one write of every population per cell update
        gbs = bpc * wl.ncell / (avg_ms * 1e-3) / 1e9
        per_set[s] = {"kernel_ms": avg_ms, "kernel_ms_median": ms[len(ms) // 2],
                      "mlups": wl.ncell / (avg_ms * 1e-3) / 1e6, "bytes_per_cell": bpc,
                      "achieved_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                      "moments_ms": sorted(mom)[len(mom) // 2],
                      "ke_log": ke_log[s][-3:]}
    dominant = max(per_set, key=lambda s: per_set[s]["kernel_ms"])
    dom = per_set[dominant]
    ncells = sum(wl.ncell for _, wl, _ in lats)
    value = ncells * a.steps / elapsed / 1e6
    tr = traffic_for(dominant, a.n)
    copy = copy_reference(dom["bytes_per_cell"] * a.n ** 3)
    roof = {"bound": "hbm", "kernel": "sl_kernel %s n=4 N=%d FP32 %d^3" % (
        dominant, 3 if dominant == "D3V27" else 2, a.n),
        "achieved": round(dom["achieved_GBs"], 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(dom["achieved_GBs"] / HBM_PEAK_GBS, 4), "traffic": tr,
        "algorithmic_bytes_per_launch": dom["bytes_per_cell"] * a.n ** 3,
        "copy_GBs": round(copy["GBs"], 1), "frac_of_copy": round(dom["achieved_GBs"] / copy["GBs"], 4)}
    out = {
        "metric": "MLUPS & %HBM peak per velocity set; adjoint/forward time; err vs FP64",
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": elapsed / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3D Taylor-Green vortex %d^3 periodic, %s, tricubic semi-Lagrangian streaming, "
                               "Courant 0.5, Ma 0.1, Re 1600, FP32, KE logged every %d steps" % (
                                   a.n, "/".join(sets), a.log_every),
                   "grid": [a.n] * 3, "sets": list(sets), "stencil": 4, "streams": nstreams},
        "per_set": {s: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
                    for s, d in per_set.items()},
        "roofline": roof,
    }
    if not a.no_extras:
        ke32 = {}
        for s, wl, lat in lats:
            ke32[s] = lat.moments(fields=False)[3].ke
        steps_done = a.warmup + a.steps + reps
        for s, wl, lat in lats:
            lat.close()
        del lats
        torch.cuda.empty_cache()
        out["err_vs_fp64"] = fp64_error(sets, a.n, steps_done, ke32)
        out["adjoint"] = adjoint_cost()
        out["large_grid"] = large_grid()
        out["svi"] = svi_throughput()
        out["svi_2048"] = svi_throughput(2048)
        out["glc"] = glc_throughput()
        out["prandtl"] = prandtl_cost()
        out["on_lattice"] = on_lattice_ratio()
        out["dissipation"] = dissipation(sets)
        torch.cuda.empty_cache()
        out["precision"] = precision_form(a.precision_n, a.precision_steps)
        torch.cuda.empty_cache()
        out["high_mach"] = high_mach(a.precision_n)
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sets, a.n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
