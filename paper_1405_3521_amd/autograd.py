"""torch.autograd wrapper: the SL fixed point V as a differentiable function of
the running cost l (the argmin controls and the reconstructed sets frozen).

    V = HJBSolve.apply(cost, problem, member, ra, opts, adj_rtol, adj_local_iters)

Forward: ``solve`` (member None) or ``solve_isa`` on the given sets, with the
policy exported.  Backward: ``adjoint`` of the policy-frozen scheme with dL/dV
routed to the owning set (``adj_local_iters`` > 0: block-asynchronous tiles);
the sets are piecewise constant in l, so they carry no gradient.  Autograd then chains through whatever produced ``cost`` (for example
l = exp(theta)).
"""
from __future__ import annotations

import dataclasses

import torch


class HJBSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cost, problem, member=None, ra=None, opts=None, adj_rtol=1e-7,
                adj_local_iters=0):
        from . import SolveOpts, solve, solve_isa
        p = dataclasses.replace(problem, cost=cost.detach().contiguous())
        o = dataclasses.replace(opts or SolveOpts(), want_policy=True)
        if member is None:
            V, pol, st = solve(p, o)
            owner = None
        else:
            V, owner, pol, _, st = solve_isa(p, ra, member, o)
        ctx.problem = p
        ctx.member = member
        ctx.owner = owner
        ctx.policy = pol
        ctx.adj_rtol = adj_rtol
        ctx.adj_local_iters = adj_local_iters
        ctx.stats = st
        return V

    @staticmethod
    def backward(ctx, dV):
        from . import adjoint
        g = dV.detach().to(ctx.problem.dtype).contiguous()
        # a negative tolerance is relative to max |g|, which the library takes on
        # the device (no host round trip here)
        dLdl, st = adjoint(ctx.problem, ctx.policy, g, ctx.member, ctx.owner,
                           tol=-ctx.adj_rtol, local_iters=ctx.adj_local_iters)
        ctx.adjoint_stats = st
        return dLdl, None, None, None, None, None, None
