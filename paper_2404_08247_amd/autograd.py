"""Differentiable radiation steps: torch.autograd.Function over the C ABI.

Forward: nsteps PD-ARS steps through rhd_step, checkpointing the state every k
steps. Backward: for each segment in reverse, rhd_step_adjoint recomputes the
segment from its checkpoint on the GPU and runs the hand-written adjoint
(transport vector-Jacobian products and an implicit-function-theorem solve at
every converged local source update). Gradients flow to the initial state and
to the Planck-mean opacity (kappa_F = kappa_P). All arithmetic runs in the
library's kernels; this module only sequences calls and holds checkpoints.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import rhd


class RHDFunction(torch.autograd.Function):
    """y_N = RHDFunction.apply(y0, kappa, solver, dt, nsteps, k).

    `solver` must be an rhd.Solver created with kappa_P = kappa (the same
    tensor), kappa_F = None and adjoint_segment_len >= k."""

    @staticmethod
    def forward(ctx, y0, kappa, solver, dt, nsteps, k):
        if kappa.data_ptr() != solver.kappa_P.data_ptr():
            raise ValueError("kappa must be the tensor the solver was created with")
        if k < 1 or k > solver.adj_len:
            raise ValueError("checkpoint interval k must be in 1..solver.adj_len")
        y = y0.detach().clone().contiguous()
        ckpts = []
        done = 0
        while done < nsteps:
            m = min(k, nsteps - done)
            ckpts.append((y.clone(), m))
            solver.step(y, dt, m)
            done += m
        ctx.solver = solver
        ctx.dt = dt
        ctx.ckpts = ckpts
        return y

    @staticmethod
    def backward(ctx, gy):
        solver = ctx.solver
        lam = gy.detach().clone().contiguous()
        gk = torch.zeros_like(solver.kappa_P)
        for state, m in reversed(ctx.ckpts):
            solver.step_adjoint(state, ctx.dt, m, lam, gk, None)
        return lam, gk, None, None, None, None


def initial_state(T: torch.Tensor, Trad: torch.Tensor, F: torch.Tensor, mom: torch.Tensor,
                  rho: torch.Tensor, params: dict) -> torch.Tensor:
    """State (E, F, E_gas, rho v) from gas and radiation temperatures, written with
    torch ops so that dJ/dT follows by the chain rule (E = a_r T_rad^4,
    E_gas = rho c_v T + |rho v|^2 / (2 rho))."""
    nd = int(params["ndim"])
    cv = params["kB_over_mu"] / (params["gamma"] - 1.0)
    E = params["a_r"] * Trad ** 4
    ke = (mom ** 2).sum(dim=0) / (2.0 * rho)
    Eg = rho * cv * T + ke
    return torch.cat([E.unsqueeze(0), F, Eg.unsqueeze(0), mom], dim=0).contiguous()


def patch_energy_gradients(params: dict, T0: torch.Tensor, mom: torch.Tensor, rho: torch.Tensor,
                           kappa: torch.Tensor, mask: torch.Tensor, dt: float, nsteps: int, k: int,
                           solver: Optional["rhd.Solver"] = None):
    """J = sum of E over `mask` after nsteps steps from T_gas = T_rad = T0, F = 0.
    Returns (J, dJ/dkappa, dJ/dT0)."""
    nd = int(params["ndim"])
    if solver is None:
        solver = rhd.Solver(params, rho, kappa, None, k, rho.device)
    T = T0.detach().clone().requires_grad_(True)
    kap = kappa if kappa.requires_grad else kappa.requires_grad_(True)
    F = torch.zeros((nd,) + tuple(T0.shape), dtype=T0.dtype, device=T0.device)
    y0 = initial_state(T, T, F, mom, rho, params)
    yN = RHDFunction.apply(y0, kap, solver, dt, nsteps, k)
    J = (yN[0] * mask).sum()
    gT, gk = torch.autograd.grad(J, [T, kap])
    return J.detach(), gk, gT
