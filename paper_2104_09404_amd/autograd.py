"""torch.autograd interface of the discrete adjoint.

``solve(u0, ...)`` returns u(T), the solution of the conservation law after nt
steps of Phi, as a differentiable function of u0.  The forward keeps only
checkpoints (every ``every``-th node); the backward runs the hand-written
reverse sweep of the library (``mgrit_adjoint``), so for
J = 1/2 ||u(T) - u_target||^2 computed with torch ops, ``J.backward()`` yields
dJ/du0 without any torch-side autodiff of the scheme.

The forward solver is either serial time stepping (``solver="serial"``) or
FAS-MGRIT (``solver="mgrit"``), whose level-0 C-points, kept with storage
mode 1, are the checkpoints (every = m).  The adjoint is that of the discrete
serial solution, which a converged MGRIT solve reproduces; an unconverged
MGRIT forward raises.
"""
from __future__ import annotations

import torch

from . import mgrit as M


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, scheme, dt, nt, every, solver, mparams, parallel_segments):
        u0c = u0.detach().contiguous()
        nx = scheme.nx
        if solver == "serial":
            ckpt = torch.empty((nt // every + 1, nx), dtype=torch.float64, device=u0.device)
            M.checkpoints(scheme, dt, nt, every, u0c, ckpt)
        elif solver == "mgrit":
            p = mparams
            if p is None:
                raise ValueError("solver='mgrit' needs mgrit parameters")
            every = p.m
            p.storage = 1
            ckpt = torch.empty((nt // every + 1, nx), dtype=torch.float64, device=u0.device)
            rc, hist, iters = M.cycle(scheme, p, u0c, ckpt)
            if rc != M.MGRIT_OK:
                raise RuntimeError("MGRIT forward did not converge (residual history %s)" % hist[-3:])
        else:
            raise ValueError("solver must be 'serial' or 'mgrit'")
        ctx.save_for_backward(ckpt)
        ctx.scheme, ctx.dt, ctx.nt, ctx.every, ctx.P = scheme, dt, nt, every, parallel_segments
        return ckpt[-1].clone()

    @staticmethod
    def backward(ctx, grad_uT):
        (ckpt,) = ctx.saved_tensors
        lam_T = grad_uT.detach().contiguous()
        lam_0 = torch.empty_like(lam_T)
        M.adjoint(ctx.scheme, ctx.dt, ctx.nt, ctx.every, ckpt, lam_T, lam_0, parallel_segments=ctx.P)
        return lam_0, None, None, None, None, None, None, None


def solve(u0: torch.Tensor, scheme: M.Scheme, dt: float, nt: int, every: int = 32, solver: str = "serial",
          mgrit_params: M.Params = None, parallel_segments: int = 0) -> torch.Tensor:
    """u(T) after nt steps from u0 (a float64 GPU tensor of nx cells), differentiable in u0."""
    return _Solve.apply(u0, scheme, dt, nt, every, solver, mgrit_params, parallel_segments)
