"""Python face of liblbm: device buffers and streams from PyTorch, every step
of the computation in the library's HIP kernels.

>>> lat = Lattice("D3Q27", (128, 128, 128), tau=0.508, order=2, stencil=4,
...               storage="f32", dx=dx, dt=dt, cs=10.0)
>>> lat.init_equilibrium(rho, u)          # torch tensors on the GPU
>>> lat.step(100)
>>> rho, u, theta, diag = lat.moments()
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import check

_STATE_DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}
_COMPUTE_DTYPE = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32, "f16": torch.float32}
_Q = {"D2Q9": 9, "D2Q19": 19, "D2Q25": 25, "D3Q13": 13, "D3Q21": 21, "D3Q27": 27, "D3V27": 27, "D3Q45": 45}
_DIM = {"D2Q9": 2, "D2Q19": 2, "D2Q25": 2, "D3Q13": 3, "D3Q21": 3, "D3Q27": 3, "D3V27": 3, "D3Q45": 3}


@dataclass
class Diagnostics:
    mass: float
    momentum: tuple
    ke: float
    energy: float
    min_rho: float
    min_theta: float
    nonfinite: int


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Lattice:
    """One semi-Lagrangian lattice Boltzmann state on one GPU."""

    def __init__(self, set: str, grid, tau: float, order: int = 2, *, stencil: int = 4, storage: str = "f32",
                 dx: float = 1.0, dt: float = 1.0, cs: float = 0.0, compressible: bool = False,
                 gamma: float = 1.4, boundary=("periodic", "periodic", "periodic"), energy_f64: bool = False,
                 support: str = "uniform", prandtl: float = 1.0, rounding: str = "nearest", seed: int = 0,
                 device=None):
        if set not in _Q:
            raise ValueError("unknown velocity set %r" % (set,))
        if storage not in _STATE_DTYPE:
            raise ValueError("unknown storage %r" % (storage,))
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self.device.type != "cuda":
            raise ValueError("liblbm runs on a GPU device")
        L = _lib.lib()
        self.set, self.storage, self.order, self.stencil = set, storage, int(order), int(stencil)
        self.D, self.Q = _DIM[set], _Q[set]
        self.A = 2 if compressible else 1
        self.compressible = bool(compressible)
        g = tuple(int(v) for v in grid) + (1,) * (3 - len(tuple(grid)))
        self.grid = g[:3]
        self.shape = (self.grid[2], self.grid[1], self.grid[0])  # (nz, ny, nx)
        self.ncell = self.grid[0] * self.grid[1] * self.grid[2]
        self.tau, self.dx, self.dt, self.gamma = float(tau), float(dx), float(dt), float(gamma)
        self.dtype = _COMPUTE_DTYPE[storage]
        self.state_dtype = _STATE_DTYPE[storage]
        opt = _lib.Options()
        L.lbm_default_options(ctypes.byref(opt))
        opt.storage = _lib.STORAGES.index(storage)
        opt.stencil = self.stencil
        opt.compressible = 1 if compressible else 0
        for a, b in enumerate(boundary):
            opt.boundary[a] = _lib.BOUNDARIES.index(b) if isinstance(b, str) else int(b)
        opt.energy_f64 = 1 if energy_f64 else 0
        opt.support = _lib.SUPPORTS.index(support)
        self.support = support
        opt.prandtl = float(prandtl)
        self.prandtl = float(prandtl)
        opt.rounding = _lib.ROUNDINGS.index(rounding)
        opt.seed = int(seed) & 0xFFFFFFFF
        self.rounding = rounding
        opt.dx, opt.dt, opt.cs, opt.gamma = self.dx, self.dt, float(cs), self.gamma
        with torch.cuda.device(self.device):
            opt.stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
            ctx = ctypes.c_void_p()
            gridarr = (ctypes.c_int64 * 3)(*self.grid)
            check(L.lbm_create(ctypes.byref(ctx), _lib.SETS.index(set), gridarr, self.tau, self.order,
                               ctypes.byref(opt)), "lbm_create")
        self._ctx = ctx
        self.cs = float(cs) if cs > 0 else self.table()["cs"]
        nbytes = int(L.lbm_state_bytes(ctx))
        elems = nbytes // torch.empty((), dtype=self.state_dtype).element_size()
        self._bufs = [torch.empty(elems, dtype=self.state_dtype, device=self.device) for _ in range(2)]
        check(L.lbm_bind(ctx, _ptr(self._bufs[0]), _ptr(self._bufs[1])), "lbm_bind")
        self.steps_taken = 0

    # -- plumbing ------------------------------------------------------------
    def _stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(_lib.lib().lbm_set_stream(self._ctx, ctypes.c_void_p(s)), "lbm_set_stream")

    def _need(self, t, shape, dtype, what):
        if t.numel() != int(torch.Size(shape).numel()):
            raise ValueError("%s: want %s elements %s, got %s" % (what, torch.Size(shape).numel(), tuple(shape),
                                                                  tuple(t.shape)))
        t = t.reshape(shape)
        if t.device != self.device or t.dtype != dtype or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
            raise ValueError("%s: want contiguous %s %s on %s, got %s %s on %s" % (
                what, dtype, tuple(shape), self.device, t.dtype, tuple(t.shape), t.device))
        return t

    @property
    def pop_shape(self):
        return (self.A * self.Q,) + self.shape

    def close(self):
        if getattr(self, "_ctx", None):
            _lib.lib().lbm_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter teardown
            pass

    def table(self):
        L = _lib.lib()
        Q, D, deg = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        cs = ctypes.c_double()
        w = (ctypes.c_double * 64)()
        xi = (ctypes.c_double * 192)()
        check(L.lbm_set_table(_lib.SETS.index(self.set), ctypes.byref(Q), ctypes.byref(D), ctypes.byref(deg),
                              ctypes.byref(cs), w, xi), "lbm_set_table")
        q = Q.value
        return {"Q": q, "D": D.value, "degree": deg.value, "cs": cs.value, "w": list(w[:q]),
                "xi": [tuple(xi[3 * i:3 * i + 3]) for i in range(q)]}

    # -- state ----------------------------------------------------------------
    def state(self):
        """The current state as a view [A*Q, nz, ny, nx] (storage dtype)."""
        p = _lib.lib().lbm_state(self._ctx)
        buf = self._bufs[0] if p == self._bufs[0].data_ptr() else self._bufs[1]
        return buf.view(self.pop_shape)

    def _state_arg(self, t, what):
        if t.dtype != self.state_dtype or not t.is_contiguous() or t.numel() != self.A * self.Q * self.ncell:
            raise ValueError("%s: want a contiguous %s tensor of %d elements, got %s %s" % (
                what, self.state_dtype, self.A * self.Q * self.ncell, t.dtype, tuple(t.shape)))
        if t.device.type not in ("cpu", "cuda"):
            raise ValueError("%s: host or GPU memory" % what)
        return t

    def get_state(self, out=None, device=None):
        """Checkpoint: a copy of the current state (lbm_get_state) into `out`
        (a contiguous tensor of the storage dtype, host or GPU), or into a new
        tensor on `device` (default: the lattice's GPU); waits for the copy."""
        if out is None:
            out = torch.empty(self.pop_shape, dtype=self.state_dtype, device=device or self.device)
        out = self._state_arg(out, "get_state")
        self._stream()
        check(_lib.lib().lbm_get_state(self._ctx, _ptr(out)), "lbm_get_state")
        return out

    def set_state(self, f):
        """Resume: copies `f` (host or GPU, storage dtype, the state's layout)
        into the current buffer (lbm_set_state); waits for the copy."""
        f = self._state_arg(f, "set_state")
        self._stream()
        check(_lib.lib().lbm_set_state(self._ctx, _ptr(f)), "lbm_set_state")

    def new_state(self):
        """A fresh device buffer shaped like the state."""
        return torch.empty(self.pop_shape, dtype=self.state_dtype, device=self.device)

    def init_equilibrium(self, rho, u, theta=None):
        self._stream()
        rho = self._need(rho, self.shape, self.dtype, "rho")
        u = self._need(u, (self.D,) + self.shape, self.dtype, "u")
        if theta is not None:
            theta = self._need(theta, self.shape, self.dtype, "theta")
        check(_lib.lib().lbm_init_equilibrium(self._ctx, _ptr(rho), _ptr(u), _ptr(theta)), "lbm_init_equilibrium")

    def step(self, n: int = 1):
        self._stream()
        check(_lib.lib().lbm_step(self._ctx, int(n)), "lbm_step")
        self.steps_taken += int(n)

    def step_into(self, src, dst):
        self._stream()
        check(_lib.lib().lbm_step_into(self._ctx, _ptr(src), _ptr(dst)), "lbm_step_into")

    def stream_only(self, src, dst):
        self._stream()
        check(_lib.lib().lbm_stream(self._ctx, _ptr(src), _ptr(dst)), "lbm_stream")

    def moments(self, state=None, fields: bool = True):
        """Per-cell rho, u, theta (compute dtype) and the diagnostics; waits for the stream."""
        self._stream()
        rho = u = th = None
        if fields:
            rho = torch.empty(self.shape, dtype=self.dtype, device=self.device)
            u = torch.empty((self.D,) + self.shape, dtype=self.dtype, device=self.device)
            th = torch.empty(self.shape, dtype=self.dtype, device=self.device)
        d = _lib.Diag()
        rc = _lib.lib().lbm_moments(self._ctx, _ptr(state), _ptr(rho), _ptr(u), _ptr(th), ctypes.byref(d))
        diag = Diagnostics(d.mass, tuple(d.momentum[:self.D]), d.ke, d.energy, d.min_rho, d.min_theta, d.nonfinite)
        check(rc, "lbm_moments")
        return rho, u, th, diag

    def enstrophy(self, u=None, order: int = 8) -> float:
        """<|curl u|^2> of the velocity field u ([D, *shape], compute dtype, as
        moments() returns it; None: the current state's), central differences
        of the given even order; waits for the stream."""
        if u is None:
            _, u, _, _ = self.moments()
        u = self._need(u, (self.D,) + self.shape, self.dtype, "u")
        self._stream()
        out = ctypes.c_double()
        check(_lib.lib().lbm_enstrophy(self._ctx, _ptr(u), int(order), ctypes.byref(out)), "lbm_enstrophy")
        return out.value

    def sync(self):
        check(_lib.lib().lbm_sync(self._ctx), "lbm_sync")

    # -- adjoint ----------------------------------------------------------------
    def adjoint_collide(self, f_prev, lam, nu):
        self._stream()
        check(_lib.lib().lbm_adjoint_collide(self._ctx, _ptr(f_prev), _ptr(lam), _ptr(nu)), "lbm_adjoint_collide")

    def adjoint_stream(self, nu, lam):
        self._stream()
        check(_lib.lib().lbm_adjoint_stream(self._ctx, _ptr(nu), _ptr(lam)), "lbm_adjoint_stream")

    def adjoint_step(self, f_prev, nu_in, nu_out):
        self._stream()
        check(_lib.lib().lbm_adjoint_step(self._ctx, _ptr(f_prev), _ptr(nu_in), _ptr(nu_out)), "lbm_adjoint_step")

    def ke_adjoint(self, f, lam):
        self._stream()
        check(_lib.lib().lbm_ke_adjoint(self._ctx, _ptr(f), _ptr(lam)), "lbm_ke_adjoint")

    def init_equilibrium_adjoint(self, rho, u, lam0, grad_u):
        self._stream()
        check(_lib.lib().lbm_init_equilibrium_adjoint(self._ctx, _ptr(rho), _ptr(u), _ptr(lam0), _ptr(grad_u)),
              "lbm_init_equilibrium_adjoint")


def stencil(set: str, dt: float, dx: float, cs: float, n: int):
    """Host-side stencil (offsets [Q][3], FP64 weights [Q][3][n]); no GPU needed."""
    import numpy as np

    Q = _Q[set]
    off = np.zeros(Q * 3, dtype=np.int32)
    w = np.zeros(Q * 3 * n, dtype=np.float64)
    check(_lib.lib().lbm_stencil(_lib.SETS.index(set), float(dt), float(dx), float(cs), int(n),
                                 off.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "lbm_stencil")
    return off.reshape(Q, 3), w.reshape(Q, 3, n)


def set_table(set: str):
    """The library's own velocity-set table (table units); no GPU needed."""
    import numpy as np

    L = _lib.lib()
    Q, D, deg = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    cs = ctypes.c_double()
    w = (ctypes.c_double * 64)()
    xi = (ctypes.c_double * 192)()
    check(L.lbm_set_table(_lib.SETS.index(set), ctypes.byref(Q), ctypes.byref(D), ctypes.byref(deg),
                          ctypes.byref(cs), w, xi), "lbm_set_table")
    q = Q.value
    return {"Q": q, "D": D.value, "degree": deg.value, "cs": cs.value, "w": np.array(w[:q]),
            "xi": np.array(xi[:3 * q]).reshape(q, 3)[:, :D.value]}
