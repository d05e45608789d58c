"""The C ABI from plain C, without Python (tests/c_abi/tgv_step.c, built by
__graft_entry__.build()): a D3Q27 FP64 Taylor-Green run of 20 steps on 32^3
through lbm_create / lbm_bind / lbm_init_equilibrium / lbm_step /
lbm_moments / lbm_enstrophy / lbm_destroy with hipMalloc'd buffers, against
the same run through the Python binding: mass, kinetic energy before and
after, and enstrophy within 1e-12 (FP64; the initial fields differ only by
the C and numpy sine and cosine).  The same program checkpoints the state to
host memory (lbm_get_state), steps on, restores it (lbm_set_state) and steps
again: the resumed run must match bit for bit."""
import math
import os
import subprocess

import numpy as np
import pytest
import torch

from paper_2101_03982_amd import Lattice

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "tgv_step")


def test_c_program_matches_python_binding():
    if not os.path.exists(EXE):
        raise RuntimeError("%s is not built; run __graft_entry__.build()" % EXE)
    run = subprocess.run([EXE, "20"], capture_output=True, text=True, timeout=120)
    assert run.returncode == 0, run.stderr
    words = run.stdout.split()
    got = {k: float(v) for k, v in zip(words[0::2], words[1::2])}
    n, u0, cs = 32, 0.05, 1.0
    dx = 2.0 * math.pi / n
    dt = 0.4 * dx / (math.sqrt(3.0) * cs)
    lat = Lattice("D3Q27", (n, n, n), 0.6, 2, stencil=4, storage="f64", dx=dx, dt=dt, cs=cs, device="cuda:0")
    x = np.arange(n) * dx
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.stack([u0 * np.sin(X) * np.cos(Y) * np.cos(Z), -u0 * np.cos(X) * np.sin(Y) * np.cos(Z), 0.0 * X])
    lat.init_equilibrium(torch.ones((n, n, n), dtype=torch.float64, device="cuda:0"),
                         torch.from_numpy(np.ascontiguousarray(u)).cuda())
    ke0 = lat.moments(fields=False)[3].ke
    lat.step(20)
    _, uu, _, d = lat.moments()
    ref = {"mass": d.mass, "ke0": ke0, "ke": d.ke, "enstrophy": lat.enstrophy(uu, order=8)}
    for key, val in ref.items():
        assert abs(got[key] / val - 1) <= 1e-12, (key, got[key], val)
    assert got["resumed_identical"] == 1 and got["stepped"] == 1, got
