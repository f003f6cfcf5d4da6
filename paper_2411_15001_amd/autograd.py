"""Reverse-mode differentiation of a rollout of the blended scheme.

`rollout(u0, nsteps, checkpoint_every, boundary=None, **params)` returns the
moments (rho, m1, m2, E) after `nsteps` steps from the initial moments u0
[4, ny, nx] (float64, device) and is differentiable with respect to u0.
`boundary` optionally maps a side (0 west, 1 east, 2 south, 3 north) to
(kinds, states) as in Solver.set_boundary: wall and Dirichlet cells, held for
the whole rollout (the Dirichlet states are constants of the map).  The backward
pass holds the blending factors theta^n and the kinetic speeds a^n at the
values of the forward pass (a fixed active set; with a fixed kinetic speed
and theta = 1 everywhere this is the exact derivative of the map).

Memory: the forward pass keeps one state every `checkpoint_every` steps;
the backward pass restores each checkpoint and recomputes its segment with
lbm_step_between, each step writing its output state into the buffer that
the next step reads and keeping its face factors theta (no state copies), then
runs the adjoint kernel step by step in reverse with those factors
(lbm_step_adjoint_theta; the same theta that lbm_step_adjoint would
recompute), and finally maps the result back through the initialisation
(lbm_init_adjoint).  All arithmetic runs in the HIP library.
"""
from __future__ import annotations

import torch

from . import binding as B
from .solver import Solver


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, nsteps, k, params, boundary):
        s = Solver(u0.detach(), **params)
        if s.params.precision != B.LBM_FP64:
            raise ValueError("the rollout adjoint is float64 only")
        for side, (kinds, states) in (boundary or {}).items():
            s.set_boundary(side, kinds, states)
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
        last = torch.empty_like(ckpts[0])  # the output of a segment's last step
        for seg in range(len(ckpts) - 1, -1, -1):
            n = min(k, nsteps - seg * k)
            # recompute the segment from its checkpoint: each step's input
            # state and its face factors; every step writes its output straight
            # into the buffer that holds the next step's input
            s.set_state(ckpts[seg])
            states, thetas = [ckpts[seg]], []
            for i in range(n):
                dst = last if i == n - 1 else torch.empty_like(ckpts[0])
                tx = torch.empty((ny, nx + 1), dtype=torch.float64, device=u0.device)
                ty = torch.empty((ny + 1, nx), dtype=torch.float64, device=u0.device)
                B.lbm_step_between(s.ctx, states[-1], dst, tx, ty)
                thetas.append((tx, ty))
                if i < n - 1:
                    states.append(dst)
            for st, (tx, ty) in zip(reversed(states), reversed(thetas)):
                B.lbm_step_adjoint_theta(s.ctx, st, tx, ty, ubar, spare)
                ubar, spare = spare, ubar
        u0bar = torch.empty_like(u0)
        B.lbm_init_adjoint(s.ctx, u0.contiguous(), ubar, u0bar)
        s.close()
        ctx.solver = None
        ctx.ckpts = None
        return u0bar, None, None, None, None


def rollout(u0, nsteps, checkpoint_every=20, boundary=None, **params):
    """Differentiable rollout: moments after nsteps steps, [4, ny, nx]."""
    return _Rollout.apply(u0, int(nsteps), int(checkpoint_every), params, boundary)
