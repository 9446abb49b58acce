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


def _mgrit_forward_params(p: M.Params, nt: int, dt: float) -> M.Params:
    """A copy of the caller's parameters with C-point storage, after checking
    that they describe the solve being differentiated: the checkpoint buffer
    holds nt/m + 1 lines of step dt, and it starts empty, so it cannot be the
    initial iterate."""
    if p.nt != nt:
        raise ValueError("mgrit_params.nt = %d differs from nt = %d" % (p.nt, nt))
    if p.dt != dt:
        raise ValueError("mgrit_params.dt = %r differs from dt = %r" % (p.dt, dt))
    if p.m < 2 or nt % p.m:
        raise ValueError("nt = %d is not a multiple of the coarsening factor m = %d" % (nt, p.m))
    if p.init != 0:
        raise ValueError("mgrit_params.init must be 0: the checkpoint buffer is not an initial iterate")
    q = M.Params.from_buffer_copy(p)
    q.storage = 1
    return q


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, scheme, dt, nt, every, solver, mparams, parallel_segments):
        u0c = u0.detach().contiguous()
        nx = scheme.nx
        if u0c.dtype != torch.float64 or u0c.numel() != nx:
            raise ValueError("u0 must hold nx = %d float64 cells" % nx)
        if nt < 1:
            raise ValueError("nt must be positive")
        if solver == "serial":
            if every < 1 or nt % every:
                raise ValueError("nt = %d is not a multiple of the checkpoint spacing %d" % (nt, every))
            ckpt = torch.empty((nt // every + 1, nx), dtype=torch.float64, device=u0.device)
            M.checkpoints(scheme, dt, nt, every, u0c, ckpt)
        elif solver == "mgrit":
            if mparams is None:
                raise ValueError("solver='mgrit' needs mgrit parameters")
            p = _mgrit_forward_params(mparams, nt, dt)
            every = p.m
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
