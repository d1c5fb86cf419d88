"""torch.autograd.Function wrappers over the HIP library (hand-written adjoints).

  FockApply          y = V_x[u] phi                    backward: fock_vjp
  FockEnergy         E_x[u]                            backward: fock_energy_vjp
  TaylorStep         psi(t+dt) = T4(-i dt h) psi(t)    backward: taylor_step_vjp
  EnergyFunctional   E[psi; A/c]                       backward: taylor_energy_vjp
  ExcitationEnergy   E[psi_t; a_t] - E[psi_0; a_0]     forward: taylor_excitation_energy
  propagate          N Taylor steps under the sin^2 pulse of Eq. (21), checkpointed every
                     `checkpoint_every` steps, returning psi(t_N) and E_ex = E(t_N) - E(t_0)

Every forward and backward computation runs in libfockmi; torch only holds
the tensors and records the graph. Gradients follow PyTorch's convention for
complex inputs (dL/dRe + i dL/dIm).
"""

from __future__ import annotations

import math

import torch
import torch.utils.checkpoint

from .api import Plan


class FockApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, phi, plan: Plan, cell: int = 0):
        ctx.plan, ctx.cell = plan, cell
        ctx.save_for_backward(u, phi)
        return plan.apply(u.contiguous(), phi.contiguous(), cell)

    @staticmethod
    def backward(ctx, g):
        u, phi = ctx.saved_tensors
        gu, gp = ctx.plan.vjp(u, phi, g.contiguous(), ctx.cell, need_u=ctx.needs_input_grad[0],
                              need_phi=ctx.needs_input_grad[1])
        return gu, gp, None, None


class FockEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, plan: Plan, cell: int = 0):
        ctx.plan, ctx.cell = plan, cell
        ctx.save_for_backward(u)
        e = plan.energy(u.contiguous(), cell)
        return torch.tensor(e.real, dtype=torch.float64)

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        return ctx.plan.energy_vjp(u.contiguous(), float(g), ctx.cell), None, None


class TaylorStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi, a_over_c, plan: Plan, dt: float, alpha: float, vloc=None, order: int = 4, cell: int = 0):
        ctx.plan, ctx.dt, ctx.alpha, ctx.vloc, ctx.order, ctx.cell = plan, dt, alpha, vloc, order, cell
        a = [float(x) for x in a_over_c.detach().cpu().reshape(3)]
        ctx.a = a
        ctx.save_for_backward(psi)
        out = psi.detach().clone().contiguous()
        plan.taylor_step(out, a, dt, alpha, vloc=vloc, order=order, cell=cell, want_norm=False)
        return out

    @staticmethod
    def backward(ctx, g):
        (psi,) = ctx.saved_tensors
        gpsi, ga = ctx.plan.taylor_step_vjp(psi.contiguous(), ctx.a, ctx.dt, ctx.alpha, g.contiguous(),
                                            vloc=ctx.vloc, order=ctx.order, cell=ctx.cell)
        return gpsi, torch.tensor(ga, dtype=torch.float64), None, None, None, None, None, None


class EnergyFunctional(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi, a_over_c, plan: Plan, alpha: float, vloc=None, cell: int = 0):
        ctx.plan, ctx.alpha, ctx.vloc, ctx.cell = plan, alpha, vloc, cell
        a = [float(x) for x in a_over_c.detach().cpu().reshape(3)]
        ctx.a = a
        ctx.save_for_backward(psi)
        e = plan.energy_functional(psi.contiguous(), a, alpha, vloc=vloc, cell=cell)
        return torch.tensor(e, dtype=torch.float64)

    @staticmethod
    def backward(ctx, g):
        (psi,) = ctx.saved_tensors
        gpsi, ga = ctx.plan.energy_functional_vjp(psi.contiguous(), ctx.a, ctx.alpha, float(g), vloc=ctx.vloc,
                                                  cell=ctx.cell)
        return gpsi, torch.tensor(ga, dtype=torch.float64), None, None, None, None


class ExcitationEnergy(torch.autograd.Function):
    """E_ex = E[psi_t; a_t] - E[psi_0; a_0] (taylor_excitation_energy: double-double
    reductions, one final rounding); backward: taylor_energy_vjp with +g and -g."""

    @staticmethod
    def forward(ctx, psi_t, a_t, psi_0, a_0, plan: Plan, alpha: float, vloc=None, cell: int = 0):
        ctx.plan, ctx.alpha, ctx.vloc, ctx.cell = plan, alpha, vloc, cell
        ctx.at = [float(x) for x in a_t.detach().cpu().reshape(3)]
        ctx.a0 = [float(x) for x in a_0.detach().cpu().reshape(3)]
        ctx.save_for_backward(psi_t, psi_0)
        e = plan.excitation_energy(psi_t.contiguous(), ctx.at, psi_0.contiguous(), ctx.a0, alpha, vloc=vloc, cell=cell)
        return torch.tensor(e, dtype=torch.float64)

    @staticmethod
    def backward(ctx, g):
        psi_t, psi_0 = ctx.saved_tensors
        gt, gat = ctx.plan.energy_functional_vjp(psi_t.contiguous(), ctx.at, ctx.alpha, float(g), vloc=ctx.vloc,
                                                 cell=ctx.cell)
        g0, ga0 = ctx.plan.energy_functional_vjp(psi_0.contiguous(), ctx.a0, ctx.alpha, -float(g), vloc=ctx.vloc,
                                                 cell=ctx.cell)
        return (gt, torch.tensor(gat, dtype=torch.float64), g0, torch.tensor(ga0, dtype=torch.float64),
                None, None, None, None)


def fock_apply(u, phi, plan, cell=0):
    return FockApply.apply(u, phi, plan, cell)


def fock_energy(u, plan, cell=0):
    return FockEnergy.apply(u, plan, cell)


def pulse_a_over_c(t, A0, omega_l, Td, direction=(0.0, 0.0, 1.0)):
    """A(t)/c of Eq. (21), A0 the amplitude of A/c (a tensor, so gradients flow to it)."""
    d = torch.tensor(direction, dtype=torch.float64)
    if 0.0 < t < Td:
        s = -math.cos(omega_l * t) * math.sin(math.pi * t / Td) ** 2
    else:
        s = 0.0
    return A0 * s * d


def propagate(plan, psi0, A0, nsteps=20, dt=0.02, alpha=0.25, omega_l=0.0569614, vloc=None, checkpoint_every=5,
              direction=(0.0, 0.0, 1.0), cell=0, order=4):
    """Taylor-propagate psi0 under the pulse of Eq. (21) with T_d = nsteps * dt.

    Returns (psi(t_N), E_ex) with E_ex = E[psi(t_N); A(t_N)/c] - E[psi0; A(0)/c]. Segments of
    `checkpoint_every` steps are recomputed in the backward pass (only their inputs are kept).
    """
    Td = nsteps * dt

    def segment(psi, A0_, s0, s1):
        for s in range(s0, s1):
            a = pulse_a_over_c(s * dt, A0_, omega_l, Td, direction)
            psi = TaylorStep.apply(psi, a, plan, dt, alpha, vloc, order, cell)
        return psi

    psi = psi0
    for s0 in range(0, nsteps, checkpoint_every):
        s1 = min(nsteps, s0 + checkpoint_every)
        if checkpoint_every < nsteps and torch.is_grad_enabled():
            psi = torch.utils.checkpoint.checkpoint(segment, psi, A0, s0, s1, use_reentrant=False)
        else:
            psi = segment(psi, A0, s0, s1)
    e_ex = ExcitationEnergy.apply(psi, pulse_a_over_c(nsteps * dt, A0, omega_l, Td, direction), psi0,
                                  pulse_a_over_c(0.0, A0, omega_l, Td, direction), plan, alpha, vloc, cell)
    return psi, e_ex
