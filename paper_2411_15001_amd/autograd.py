"""Reverse-mode differentiation of a rollout of the blended scheme.

`rollout(u0, nsteps, checkpoint_every, **params)` returns the moments
(rho, m1, m2, E) after `nsteps` steps from the initial moments u0 [4, ny, nx]
(float64, device) and is differentiable with respect to u0.  The backward
pass holds the blending factors theta^n and the kinetic speeds a^n at the
values of the forward pass (a fixed active set; with a fixed kinetic speed
and theta = 1 everywhere this is the exact derivative of the map).

Memory: the forward pass keeps one state every `checkpoint_every` steps;
the backward pass restores each checkpoint, recomputes its segment keeping
the segment's states, and runs the adjoint kernel step by step in reverse
(lbm_step_adjoint), then maps the result back through the initialisation
(lbm_init_adjoint).  All arithmetic runs in the HIP library.
"""
from __future__ import annotations

import torch

from . import binding as B
from .solver import Solver


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, nsteps, k, params):
        s = Solver(u0.detach(), **params)
        if s.params.precision != B.LBM_FP64:
            raise ValueError("the rollout adjoint is float64 only")
        ckpts = [s.get_state()]
        done = 0
        while done < nsteps:
            n = min(k, nsteps - done)
            s.step(n)
            done += n
            if done < nsteps:
                ckpts.append(s.get_state())
        out = s.moments()
        ctx.solver = s
        ctx.ckpts = ckpts
        ctx.nsteps = nsteps
        ctx.k = k
        ctx.save_for_backward(u0)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        (u0,) = ctx.saved_tensors
        s, ckpts, nsteps, k = ctx.solver, ctx.ckpts, ctx.nsteps, ctx.k
        ny, nx = s.ny, s.nx
        ubar = torch.zeros((20, ny, nx), dtype=torch.float64, device=u0.device)
        ubar[0:4] = grad_out.to(torch.float64)
        spare = torch.empty_like(ubar)
        for seg in range(len(ckpts) - 1, -1, -1):
            n = min(k, nsteps - seg * k)
            # recompute the segment's states from its checkpoint
            states = [ckpts[seg]]
            s.set_state(ckpts[seg])
            for _ in range(n - 1):
                s.step(1)
                states.append(s.get_state())
            for st in reversed(states):
                B.lbm_step_adjoint(s.ctx, st, ubar, spare)
                ubar, spare = spare, ubar
        u0bar = torch.empty_like(u0)
        B.lbm_init_adjoint(s.ctx, u0.contiguous(), ubar, u0bar)
        s.close()
        ctx.solver = None
        ctx.ckpts = None
        return u0bar, None, None, None


def rollout(u0, nsteps, checkpoint_every=20, **params):
    """Differentiable rollout: moments after nsteps steps, [4, ny, nx]."""
    return _Rollout.apply(u0, int(nsteps), int(checkpoint_every), params)
