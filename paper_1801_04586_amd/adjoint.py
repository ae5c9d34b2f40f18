"""Gradients of a flow loss through the cascaded-LBM time loop.

``flow_loss(force_field, rates, lattice, state0, u_target, nsteps, K)`` returns
J = 1/2 sum_fluid |u(x, T) - u_target(x)|^2 after T = nsteps steps of the
lattice started from ``state0``, with the per-node body-force field and the ten
relaxation rates of Eq. (13) as differentiable inputs.  The backward pass runs
the hand-written adjoint kernels (``clbm_loss_seed``, ``clbm_adjoint_step``):

  * forward: T steps through clbm_run (fused step pairs where it uses them),
    a copy of the state kept every K steps (checkpoints);
  * backward: segments from last to first; the K - 1 states after a
    segment's checkpoint are recomputed from it by clbm_trajectory (single
    steps, bitwise identical to the original run, whose fused pairs are
    bitwise two single steps), then the adjoint steps walk back through the
    checkpoint and those states.

Memory: ceil(T/K) checkpoints + K - 1 segment states + two adjoint buffers.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .clbm import Lattice


class _FlowLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, force_field, rates, lat: Lattice, state0, u_target, nsteps: int, K: int):
        nsteps, K = int(nsteps), int(K)
        if nsteps < 0 or K < 1:
            raise ValueError("nsteps >= 0 and K >= 1 required")
        field = force_field.detach().to(device=lat.device, dtype=lat.real).contiguous()
        lat.set_force(lat.force, field, lat.force_scale)
        rate_values = rates.detach().cpu().to(torch.float64).numpy().copy()
        lat.set_rates(rate_values)
        c = lat.ctx
        a, b = torch.empty_like(state0), torch.empty_like(state0)
        c.copy(state0, a)
        ckpts = []
        t = 0
        while t < nsteps:  # a checkpoint every K steps; clbm_run may fuse the steps in between
            ck = torch.empty_like(a)
            c.copy(a, ck)
            ckpts.append(ck)
            n = min(K, nsteps - t)
            if c.run(a, b, n):
                a, b = b, a
            t += n
        ut = u_target.detach().to(device=lat.device, dtype=lat.real).contiguous()
        lam = torch.empty((27,) + lat.shape, dtype=lat.real, device=lat.device)
        dJdF = torch.zeros((3,) + lat.shape, dtype=lat.real, device=lat.device)
        J = torch.zeros(1, dtype=torch.float64, device=lat.device)
        c.loss_seed(a, ut, lam, dJdF, J)
        ctx.lat, ctx.nsteps, ctx.K = lat, nsteps, K
        ctx.ckpts, ctx.lam, ctx.dJdF = ckpts, lam, dJdF
        ctx.field = field
        # the lattice may be reconfigured before backward runs: keep what this forward pass used
        ctx.rates, ctx.force, ctx.force_scale = rate_values, lat.force, lat.force_scale
        ctx.rates_meta = (rates.dtype, rates.device)
        ctx.ff_meta = (force_field.dtype, force_field.device)
        return J[0]

    @staticmethod
    def backward(ctx, gJ):
        lat, nsteps, K = ctx.lat, ctx.nsteps, ctx.K
        c = lat.ctx
        lat.set_force(ctx.force, ctx.field, ctx.force_scale)
        lat.set_rates(ctx.rates)
        lam, dJdF = ctx.lam, ctx.dJdF
        lam2 = torch.empty_like(lam)
        dJds = torch.zeros(10, dtype=torch.float64, device=lat.device)
        nseg = len(ctx.ckpts)
        seg = [torch.empty_like(ctx.ckpts[0]) for _ in range(min(K, nsteps) - 1)] if nseg else []
        for sidx in range(nseg - 1, -1, -1):
            t0 = sidx * K
            t1 = min(t0 + K, nsteps)
            states = [ctx.ckpts[sidx]] + seg[: t1 - t0 - 1]  # states at t0 ... t1 - 1
            c.trajectory(states[0], states[1:])
            for t in range(t1 - 1, t0 - 1, -1):
                c.adjoint_step(states[t - t0], lam, lam2, dJdF, dJds)
                lam, lam2 = lam2, lam
        g = gJ.to(torch.float64)
        # the kernels accumulate dJ/dF for the total force F = uniform + force_scale * field
        gF = (dJdF.to(torch.float64) * (g * ctx.force_scale)).to(dtype=ctx.ff_meta[0], device=ctx.ff_meta[1])
        gs = (dJds * g).to(dtype=ctx.rates_meta[0], device=ctx.rates_meta[1])
        ctx.ckpts = None
        return gF, gs, None, None, None, None, None


def flow_loss(force_field: torch.Tensor, rates: torch.Tensor, lat: Lattice, state0: torch.Tensor,
              u_target: torch.Tensor, nsteps: int, K: int = 20) -> torch.Tensor:
    """J(F, s) with adjoint gradients; see the module docstring."""
    return _FlowLoss.apply(force_field, rates, lat, state0, u_target, nsteps, K)


def initial_gradient(lat: Lattice, state0: torch.Tensor, u_target: torch.Tensor, nsteps: int):
    """(J, dJ/df(0)) for the current force and rates, storing every state (for tests)."""
    c = lat.ctx
    states = [state0]
    for _ in range(int(nsteps)):
        nxt = torch.empty_like(state0)
        c.step(states[-1], nxt)
        states.append(nxt)
    lam = torch.empty((27,) + lat.shape, dtype=lat.real, device=lat.device)
    lam2 = torch.empty_like(lam)
    J = torch.zeros(1, dtype=torch.float64, device=lat.device)
    ut = u_target.detach().to(device=lat.device, dtype=lat.real).contiguous()
    c.loss_seed(states[-1], ut, lam, None, J)
    for t in range(int(nsteps) - 1, -1, -1):
        c.adjoint_step(states[t], lam, lam2, None, None)
        lam, lam2 = lam2, lam
    return float(J.item()), lam


def checkpoint_memory_bytes(lat: Lattice, nsteps: int, K: int) -> int:
    per = lat.state.numel() * lat.state.element_size()
    return (math.ceil(nsteps / K) + K - 1) * per
