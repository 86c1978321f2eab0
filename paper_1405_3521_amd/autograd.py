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

# Workspaces kept across calls, one per (device, stage): a repeated forward or
# backward then hands the library the same device addresses, so it replays its
# captured sweep graphs and polls on the previous call's schedule instead of
# capturing anew.  Calls are ordered on the current stream, so a later call
# reuses a workspace only after the earlier call's kernels.
_WORKSPACES = {}


def _workspace(stage, nbytes, device):
    key = (str(device), stage)
    ws = _WORKSPACES.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
        _WORKSPACES[key] = ws
    return ws


class HJBSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cost, problem, member=None, ra=None, opts=None, adj_rtol=1e-7,
                adj_local_iters=0):
        from . import SolveOpts, isa_workspace_bytes, solve, solve_isa, solve_workspace_bytes
        p = dataclasses.replace(problem, cost=cost.detach().contiguous())
        o = dataclasses.replace(opts or SolveOpts(), want_policy=True)
        dev = p.target.device
        if member is None:
            ws = _workspace("solve", solve_workspace_bytes(p), dev)
            V, pol, st = solve(p, o, workspace=ws)
            owner = None
        else:
            ws = _workspace("isa", isa_workspace_bytes(p, ra), dev)
            V, owner, pol, _, st = solve_isa(p, ra, member, o, workspace=ws)
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
        from . import adjoint, adjoint_workspace_bytes
        g = dV.detach().to(ctx.problem.dtype).contiguous()
        n_sets = ctx.problem.n_comp if ctx.member is not None else 1
        ws = _workspace("adjoint", adjoint_workspace_bytes(ctx.problem, n_sets), g.device)
        # a negative tolerance is relative to max |g|, which the library takes on
        # the device (no host round trip here)
        dLdl, st = adjoint(ctx.problem, ctx.policy, g, ctx.member, ctx.owner,
                           tol=-ctx.adj_rtol, local_iters=ctx.adj_local_iters, workspace=ws)
        ctx.adjoint_stats = st
        return dLdl, None, None, None, None, None, None
