"""ctypes binding of the plain FP64 CPU oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It never touches the
GPU library, and the GPU library never touches it.

Every function takes and returns float64 numpy arrays in the layout
``[A*Q][nz][ny][nx]`` (populations) or ``[D][nz][ny][nx]`` (velocities), x
fastest.  The C source cites, per function, the passage of the paper it
follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

SETS = ["D2Q9", "D2Q19", "D2Q25", "D3Q13", "D3Q21", "D3Q27", "D3V27", "D3Q45"]
PERIODIC, EXTRAPOLATE = 0, 1
# streaming support: uniform grid with an n-node Lagrange stencil, or the
# paper's cell-wise interpolation on Gauss-Lobatto-Chebyshev points
# (cells of p = stencil - 1 intervals; periodic axes whose extents are
# multiples of p)
KINDS = ("uniform", "glc")

GCC_FLAGS = ["-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("set", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("stencil", ctypes.c_int32),
        ("compressible", ctypes.c_int32),
        ("nx", ctypes.c_int64),
        ("ny", ctypes.c_int64),
        ("nz", ctypes.c_int64),
        ("bc", ctypes.c_int32 * 3),
        ("kind", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("cs", ctypes.c_double),
        ("tau", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("prandtl", ctypes.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB points the tests at a deliberately broken copy of the
        # oracle (tests/test_oracle_mutants.py); normally unset.
        path = os.environ.get("ORACLE_LIB") or build()
        _lib = ctypes.CDLL(path)
        _lib.orc_num_threads.restype = ctypes.c_int
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _arr(a, dtype=np.float64):
    return np.ascontiguousarray(a, dtype=dtype)


@dataclass
class Config:
    """Problem description shared by every oracle call."""

    set: str
    grid: tuple  # (nx, ny, nz); nz = 1 in 2D
    tau: float
    order: int = 2
    stencil: int = 3
    dx: float = 1.0
    dt: float = 1.0
    cs: float = 0.0  # <= 0: the set's own tabulated speed of sound
    compressible: bool = False
    gamma: float = 1.4
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)
    kind: str = "uniform"
    prandtl: float = 1.0  # compressible model: heat fluxes relaxed for this Prandtl number
    _c: _Cfg = field(default=None, repr=False)

    def __post_init__(self):
        c = _Cfg()
        c.set = SETS.index(self.set)
        c.order = int(self.order)
        c.stencil = int(self.stencil)
        c.compressible = 1 if self.compressible else 0
        nx, ny, nz = (tuple(self.grid) + (1, 1))[:3]
        c.nx, c.ny, c.nz = int(nx), int(ny), int(nz)
        for a in range(3):
            c.bc[a] = int(self.bc[a])
        c.kind = KINDS.index(self.kind)
        c.dx, c.dt, c.cs, c.tau, c.gamma = (float(self.dx), float(self.dt), float(self.cs),
                                            float(self.tau), float(self.gamma))
        c.prandtl = float(self.prandtl)
        self._c = c
        self.D = table(self.set)["D"]
        self.Q = table(self.set)["Q"]
        self.A = 2 if self.compressible else 1

    @property
    def ref(self):
        return ctypes.byref(self._c)

    @property
    def shape(self):
        nx, ny, nz = (tuple(self.grid) + (1, 1))[:3]
        return (nz, ny, nx) if self.D == 3 else (1, ny, nx)

    @property
    def ncell(self):
        return int(np.prod(self.shape))

    def pop_shape(self):
        return (self.A * self.Q,) + self.shape


def table(name: str) -> dict:
    """The oracle's own velocity set, in table units (before rescaling)."""
    Q = ctypes.c_int32()
    D = ctypes.c_int32()
    deg = ctypes.c_int32()
    cs = ctypes.c_double()
    w = np.zeros(64)
    xi = np.zeros((64, 3))
    rc = lib().orc_set_table(SETS.index(name), ctypes.byref(Q), ctypes.byref(D), ctypes.byref(deg),
                             ctypes.byref(cs), _p(w), _p(xi))
    if rc:
        raise ValueError(name)
    q = Q.value
    return {"Q": q, "D": D.value, "degree": deg.value, "cs": cs.value, "w": w[:q].copy(),
            "xi": xi[:q, :D.value].copy()}


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("oracle %s failed (%d)" % (what, rc))


def init(cfg: Config, rho, u, theta=None):
    rho = _arr(rho).reshape(cfg.shape)
    u = _arr(u).reshape((cfg.D,) + cfg.shape)
    th = None if theta is None else _arr(theta).reshape(cfg.shape)
    f = np.empty(cfg.pop_shape())
    _check(lib().orc_init(cfg.ref, _p(rho), _p(u), None if th is None else _p(th), _p(f)), "init")
    return f


def stream(cfg: Config, f):
    f = _arr(f)
    out = np.empty_like(f)
    _check(lib().orc_stream(cfg.ref, _p(f), _p(out)), "stream")
    return out


def stream_transpose(cfg: Config, mu):
    mu = _arr(mu)
    out = np.empty_like(mu)
    _check(lib().orc_stream_transpose(cfg.ref, _p(mu), _p(out)), "stream_transpose")
    return out


def collide(cfg: Config, ft):
    ft = _arr(ft)
    out = np.empty_like(ft)
    _check(lib().orc_collide(cfg.ref, _p(ft), _p(out)), "collide")
    return out


def step(cfg: Config, f):
    f = _arr(f)
    out = np.empty_like(f)
    tmp = np.empty_like(f)
    _check(lib().orc_step(cfg.ref, _p(f), _p(out), _p(tmp)), "step")
    return out


def run(cfg: Config, f, nsteps: int):
    f = _arr(f).copy()
    scratch = np.empty((2,) + f.shape)
    _check(lib().orc_run(cfg.ref, _p(f), ctypes.c_int64(int(nsteps)), _p(scratch)), "run")
    return f


def moments(cfg: Config, f):
    """Per-cell rho, u (physical units), theta, and the diagnostics dict."""
    f = _arr(f)
    rho = np.empty(cfg.shape)
    u = np.empty((cfg.D,) + cfg.shape)
    th = np.empty(cfg.shape)
    d = np.empty(8)
    _check(lib().orc_moments(cfg.ref, _p(f), _p(rho), _p(u), _p(th), _p(d)), "moments")
    diag = {"mass": d[0], "momentum": d[1:1 + cfg.D].copy(), "ke": d[4], "energy": d[5],
            "min_rho": d[6], "min_theta": d[7]}
    return rho, u, th, diag


def feq(cfg: Config, rho: float, u, theta: float = 1.0):
    u = _arr(np.asarray(u, dtype=np.float64).ravel()[:cfg.D])
    out = np.empty(cfg.A * cfg.Q)
    _check(lib().orc_feq(cfg.ref, ctypes.c_double(rho), _p(u), ctypes.c_double(theta), _p(out)), "feq")
    return out


def collide_one(cfg: Config, fin):
    fin = _arr(fin)
    out = np.empty_like(fin)
    _check(lib().orc_collide_one(cfg.ref, _p(fin), _p(out)), "collide_one")
    return out


def collide_jacobian(cfg: Config, fin):
    fin = _arr(fin)
    n = fin.size
    J = np.empty((n, n))
    _check(lib().orc_collide_jacobian(cfg.ref, _p(fin), _p(J)), "collide_jacobian")
    return J


def adjoint_collide(cfg: Config, ft, lam):
    ft, lam = _arr(ft), _arr(lam)
    out = np.empty_like(ft)
    _check(lib().orc_adjoint_collide(cfg.ref, _p(ft), _p(lam), _p(out)), "adjoint_collide")
    return out


def ke_and_grad(cfg: Config, f, want_grad: bool = True):
    f = _arr(f)
    ke = ctypes.c_double()
    g = np.empty_like(f) if want_grad else None
    _check(lib().orc_ke_and_grad(cfg.ref, _p(f), ctypes.byref(ke), None if g is None else _p(g)), "ke")
    return ke.value, g


def init_transpose(cfg: Config, rho, u, lam0, theta=None):
    rho = _arr(rho).reshape(cfg.shape)
    u = _arr(u).reshape((cfg.D,) + cfg.shape)
    lam0 = _arr(lam0)
    th = None if theta is None else _arr(theta).reshape(cfg.shape)
    g = np.empty((cfg.D,) + cfg.shape)
    _check(lib().orc_init_transpose(cfg.ref, _p(rho), _p(u), None if th is None else _p(th), _p(lam0), _p(g)),
           "init_transpose")
    return g


def ke_gradient_u0(cfg: Config, rho, u, nsteps: int, theta=None):
    """Loss (mean kinetic energy after nsteps) and its gradient w.r.t. u0."""
    rho = _arr(rho).reshape(cfg.shape)
    u = _arr(u).reshape((cfg.D,) + cfg.shape)
    th = None if theta is None else _arr(theta).reshape(cfg.shape)
    loss = ctypes.c_double()
    g = np.empty((cfg.D,) + cfg.shape)
    _check(lib().orc_ke_gradient_u0(cfg.ref, _p(rho), _p(u), None if th is None else _p(th),
                                    ctypes.c_int64(int(nsteps)), ctypes.byref(loss), _p(g)), "ke_gradient_u0")
    return loss.value, g


def first_step_at(cfg: Config, rho, u, cells, theta=None):
    """One step from the equilibrium of (rho, u, theta), evaluated only at the
    flat cell indices ``cells``; returns [len(cells)][A*Q]."""
    rho = _arr(rho).reshape(cfg.shape)
    u = _arr(u).reshape((cfg.D,) + cfg.shape)
    th = None if theta is None else _arr(theta).reshape(cfg.shape)
    cells = _arr(cells, np.int64).ravel()
    out = np.empty((cells.size, cfg.A * cfg.Q))
    _check(lib().orc_first_step_at(cfg.ref, _p(rho), _p(u), None if th is None else _p(th), _p(cells),
                                   ctypes.c_int64(cells.size), _p(out)), "first_step_at")
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())
