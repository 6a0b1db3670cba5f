"""Differentiable rollout: the loss of a fixed-geometry run as a function of
the initial density of component A, the Shan-Chen coupling G and the body
acceleration g, with gradients from the library's reverse sweep (lb_backward).

The forward pass runs `steps` steps of the HIP path from f = f_eq(rho0, 0)
(Eq. LEQ), recording a checkpoint every `checkpoint_every` steps, and
evaluates L = sum over fluid nodes of |3 sum_i w_i phi(n + c_i) c_i|^2 with
phi = psi_A - psi_B on the final state. The backward pass recomputes each
segment from its checkpoint and runs the adjoint kernels through it. Spheres
are static obstacles (their map is constant, so L is differentiable).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import torch

from .lattice import Lattice, Params


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rhoA0, G, g, rhoB0, params: Params, steps: int, x, checkpoint_every: int):
        p = dataclasses.replace(params, G=float(G), g=tuple(float(v) for v in g.tolist()),
                                checkpoint_every=int(checkpoint_every),
                                max_record_steps=int(steps), particles_fixed=True,
                                max_particles=0 if x is None else int(len(x)))
        rho = [rhoA0.detach().to("cpu", torch.float64).numpy().reshape(-1)]
        if p.ncomp == 2:
            rho.append(rhoB0.detach().to("cpu", torch.float64).numpy().reshape(-1))
        lat = Lattice(p, np.stack(rho))
        if x is not None and len(x):
            lat.add_particles(np.asarray(x, dtype=np.float64))
        lat.step(steps)
        L, sA, sB = lat.loss(seeds=True)
        ctx.lat, ctx.seeds = lat, (sA, sB)
        ctx.shape, ctx.device = rhoA0.shape, rhoA0.device
        return torch.tensor(L, dtype=torch.float64, device=rhoA0.device)

    @staticmethod
    def backward(ctx, gL):
        lat = ctx.lat
        sA, sB = ctx.seeds
        dA0, dG, dg = lat.backward(sA, sB if lat.params.ncomp == 2 else None)
        lat.close()
        ctx.lat = ctx.seeds = None
        gA = gL * dA0.to(ctx.device).reshape(ctx.shape)
        gG = gL * torch.tensor(dG, dtype=torch.float64, device=ctx.device)
        gg = gL * torch.tensor(dg, dtype=torch.float64, device=ctx.device)
        return gA, gG, gg, None, None, None, None, None


def rollout_loss(params: Params, rhoA0: torch.Tensor, G: torch.Tensor, g: torch.Tensor,
                 rhoB0: Optional[torch.Tensor] = None, steps: int = 500,
                 x: Optional[np.ndarray] = None, checkpoint_every: int = 50) -> torch.Tensor:
    """L after `steps` steps; differentiable in rhoA0 ([N] or [nz, ny, nx],
    node order x fastest), G (0-d) and g ([3]). FP64 scalar tensor."""
    if rhoB0 is None:
        rhoB0 = torch.ones_like(rhoA0)
    return _Rollout.apply(rhoA0, G, g, rhoB0, params, steps, x, checkpoint_every)
