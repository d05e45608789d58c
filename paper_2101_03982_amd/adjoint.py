"""Reverse-mode derivative of a semi-Lagrangian lattice Boltzmann rollout.

``KineticEnergyRollout`` is a ``torch.autograd.Function`` mapping the initial
velocity field u0 (density rho0 fixed) to the mean kinetic energy after T
steps, K = <|u(T)|^2 / 2>.  Forward: f_0 = f^eq(rho0, u0), f_{t+1} = C(S f_t),
keeping a checkpoint every ``every`` steps.  Backward, segment by segment in
reverse: recompute the segment's states from its checkpoint, then run the
library's adjoint kernels backwards through them:
  lam_T = dK/df_T;  nu_T = J_C(S f_{T-1})^T lam_T;
  nu_t  = J_C(S f_{t-1})^T S^T nu_{t+1}  (fused kernel);
  lam_0 = S^T nu_1;  dK/du0 = (d f^eq / d u0)^T lam_0.
Every arithmetic step runs in the library's HIP kernels.
"""
from __future__ import annotations

import torch

from .lattice import Lattice


def rollout_states(lat: Lattice, f0, steps: int):
    """All states f_0 .. f_steps as a list of tensors (for small problems)."""
    out = [f0.clone()]
    for _ in range(steps):
        nxt = lat.new_state()
        lat.step_into(out[-1], nxt)
        out.append(nxt)
    return out


class KineticEnergyRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, rho0, lat: Lattice, steps: int, every: int):
        if steps < 1 or every < 1:
            raise ValueError("steps and every must be positive")
        lat.init_equilibrium(rho0, u0)
        f = lat.state().clone()
        ckpts = {0: f.clone()}
        a, b = f, lat.new_state()
        for t in range(steps):
            lat.step_into(a, b)
            a, b = b, a
            if (t + 1) % every == 0 and t + 1 < steps:
                ckpts[t + 1] = a.clone()
        _, _, _, diag = lat.moments(a, fields=False)
        ctx.lat, ctx.steps, ctx.every = lat, steps, every
        ctx.ckpts = ckpts
        ctx.f_T = a.clone()
        ctx.save_for_backward(u0, rho0)
        return torch.tensor(diag.ke, dtype=torch.float64, device=u0.device)

    @staticmethod
    def backward(ctx, gK):
        lat: Lattice = ctx.lat
        u0, rho0 = ctx.saved_tensors
        T, K = ctx.steps, ctx.every
        lam = lat.new_state()
        lat.ke_adjoint(ctx.f_T, lam)
        lam.mul_(gK.to(lam.dtype))
        nu, nu_next = lat.new_state(), lat.new_state()
        have_nu = False
        starts = sorted(ctx.ckpts.keys())
        for s in reversed(starts):
            e = min(s + K, T)  # states f_s .. f_{e-1} start the steps s+1 .. e
            seg = [ctx.ckpts[s]]
            for _ in range(s + 1, e):
                nxt = lat.new_state()
                lat.step_into(seg[-1], nxt)
                seg.append(nxt)
            for t in range(e, s, -1):  # step t maps f_{t-1} -> f_t
                f_prev = seg[t - 1 - s]
                if not have_nu:
                    lat.adjoint_collide(f_prev, lam, nu)
                    have_nu = True
                else:
                    lat.adjoint_step(f_prev, nu, nu_next)
                    nu, nu_next = nu_next, nu
            del seg
        lat.adjoint_stream(nu, lam)
        grad = torch.empty_like(u0)
        lat.init_equilibrium_adjoint(rho0, u0, lam, grad)
        return grad, None, None, None, None


def kinetic_energy_after(u0, rho0, lat: Lattice, steps: int, every: int = 20):
    """K(u0) = <|u(T)|^2/2> after ``steps`` steps; differentiable in u0."""
    return KineticEnergyRollout.apply(u0, rho0, lat, steps, every)
