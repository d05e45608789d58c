"""Shared helpers of the GPU tests: build the GPU lattice and the oracle
configuration of one problem from the same parameters, and compare states.

Set LBM_PARITY_LOG to a file name to have the parity tests append the errors
they measured (one JSON object per line), beside asserting their bounds."""
import json
import os

import numpy as np
import torch

from paper_2101_03982_amd import Lattice

BC = {0: "periodic", 1: "extrapolate"}


def pair(orc, set_, grid, tau, order=2, n=4, storage="f64", dx=1.0, dt=1.0, cs=0.0, compressible=False,
         gamma=1.4, bc=(0, 0, 0), energy_f64=False, support="uniform", prandtl=1.0, rounding="nearest", seed=0):
    """(GPU lattice, oracle config) of the same problem (rounding and seed:
    the GPU's storage only)."""
    lat = Lattice(set_, grid, tau, order, stencil=n, storage=storage, dx=dx, dt=dt, cs=cs,
                  compressible=compressible, gamma=gamma, boundary=tuple(BC[b] for b in bc), energy_f64=energy_f64,
                  support=support, prandtl=prandtl, rounding=rounding, seed=seed, device="cuda:0")
    cfg = orc.Config(set_, tuple(grid) + (1,) * (3 - len(grid)), tau=tau, order=order, stencil=n, dx=dx, dt=dt,
                     cs=cs, compressible=compressible, gamma=gamma, bc=bc, kind=support, prandtl=prandtl)
    return lat, cfg


def to_dev(a, dtype):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0", dtype)


def init_both(lat, orc, cfg, rho, u, theta=None):
    lat.init_equilibrium(to_dev(rho, lat.dtype), to_dev(u, lat.dtype), to_dev(theta, lat.dtype))
    return orc.init(cfg, rho, u, theta)


def gpu_populations(lat, state=None):
    """The state as float64 numpy populations (deviation storage adds back the
    reference values w_i and (2 C_v - D) w_i)."""
    f = (lat.state() if state is None else state).to(torch.float64).cpu().numpy()
    if lat.storage in ("f32", "bf16", "f16"):
        t = lat.table()
        w = np.array(t["w"])
        ref = [w]
        if lat.A == 2:
            Cv = 1.0 / (lat.gamma - 1.0)
            ref.append((2 * Cv - lat.D) * w)
        f = f + np.concatenate(ref).reshape((-1,) + (1,) * 3)
    return f


def rel_err(a, b):
    """max |a - b| / max |b|."""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def reference_values(lat):
    """r_i per stored array, [A*Q]: w_i for f and (2 C_v - D) w_i for g (the
    values deviation storage subtracts)."""
    w = np.array(lat.table()["w"])
    ref = [w]
    if lat.A == 2:
        ref.append((2.0 / (lat.gamma - 1.0) - lat.D) * w)
    return np.concatenate(ref)


def pop_err(lat, got, ref, axis=0):
    """Largest error of any population relative to that population's own
    scale: max over populations k of max_cells |got_k - ref_k| divided by
    max_cells |ref_k - r_k|, r_k its reference value (reference_values).
    Small-weight populations then count as much as the large ones.  `axis`
    is the population axis of got and ref."""
    r = reference_values(lat)
    got = np.moveaxis(np.asarray(got, dtype=np.float64), axis, 0).reshape(len(r), -1)
    ref = np.moveaxis(np.asarray(ref, dtype=np.float64), axis, 0).reshape(len(r), -1)
    scale = np.max(np.abs(ref - r[:, None]), axis=1)
    err = np.max(np.abs(got - ref), axis=1)
    return float(np.max(err / np.maximum(scale, 1e-300)))


def note(case, **values):
    """Appends the measured errors of a parity case to $LBM_PARITY_LOG."""
    path = os.environ.get("LBM_PARITY_LOG")
    if path:
        with open(path, "a") as fh:
            fh.write(json.dumps({"case": case, **{k: float(v) for k, v in values.items()}}) + "\n")
