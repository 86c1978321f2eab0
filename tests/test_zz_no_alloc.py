"""The no-allocation entry point (sl_solve_noalloc) against sl_solve, through the
C ABI: the same global solve with the library's static device scratch in place of
a caller workspace.  Both run the same kernels with the same arguments, so the
values and policies must agree bit for bit, on two calls in a row (the second on
a smaller grid, so the scratch holds the first call's data when it starts)."""
import numpy as np
import pytest
import torch

import paper_1405_3521_amd as S
import workloads as W

pytestmark = pytest.mark.gpu

CAP = 50_000


def say(*a):
    print(*a, flush=True)


def _pair(p, dtype, opts):
    dp = S.to_device(p, dtype)
    V_ref, pol_ref, st_ref = S.solve(dp, opts)
    V, pol, st = S.solve_noalloc(dp, opts)
    torch.cuda.synchronize()
    return (V_ref.cpu().numpy(), None if pol_ref is None else pol_ref.cpu().numpy(), st_ref,
            V.cpu().numpy(), None if pol is None else pol.cpu().numpy(), st)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("local", [0, 8])
def test_noalloc_equals_solve_two_calls(dtype, local):
    opts = S.SolveOpts(tol=0.0, max_sweeps=CAP, want_policy=True, local_iters=local)
    for p in (W.c2_multitarget(n=193, m=32), W.c2_multitarget(n=65, m=16)):
        say("case: noalloc", p.name, p.n, dtype, "local", local)
        V_ref, pol_ref, st_ref, V, pol, st = _pair(p, dtype, opts)
        assert st["converged"] and st_ref["converged"]
        assert np.array_equal(V, V_ref), np.abs(V.astype(np.float64) - V_ref).max()
        assert np.array_equal(pol, pol_ref)
        assert st["sweeps_max"] == st_ref["sweeps_max"]
        assert st["node_control_updates"] == st_ref["node_control_updates"]


def test_noalloc_with_cost_drift_and_tolerance_stop():
    """Fields that take scratch beyond the value buffers (scaled cost, drift in
    index units) and a stop at a tolerance: the same iterate as sl_solve."""
    p = W.c5_adjoint(n=129, n_obs=100, swirl=0.5)
    opts = S.SolveOpts(tol=1e-6, max_sweeps=CAP, local_iters=4)
    say("case: noalloc cost+drift", p.n)
    V_ref, _, st_ref, V, _, st = _pair(p, torch.float32, opts)
    assert np.array_equal(V, V_ref)
    assert st["sweeps_max"] == st_ref["sweeps_max"]
    q = W.c1_eikonal(51)
    say("case: noalloc eikonal after", q.n)
    V_ref, _, _, V, _, _ = _pair(q, torch.float64, S.SolveOpts(tol=0.0, max_sweeps=CAP))
    assert np.array_equal(V, V_ref)


def test_noalloc_rejects_oversize_and_timing_options():
    p = W.c2_multitarget(n=2049, m=8)
    dp = S.to_device(p, torch.float32)
    with pytest.raises(S.SlError) as e:
        S.solve_noalloc(dp, S.SolveOpts(tol=1e-3, max_sweeps=10))
    assert e.value.status == -6
    q = S.to_device(W.c1_eikonal(33), torch.float32)
    for bad in (S.SolveOpts(autotune=1), S.SolveOpts(profile=True)):
        with pytest.raises(S.SlError) as e:
            S.solve_noalloc(q, bad)
        assert e.value.status == -1
