"""The Kruzkov form of the weighted minimum-time problem (per-node discount
exp(-h l_j), disc = "kruzkov") on the GPU against the oracle: FP64 bit-exact,
FP32 within 1e-5, sets and labels bit-exact, block-asynchronous sweeps equal to
Jacobi bit for bit."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1405_3521_amd as S
import workloads as W
from oracle import isa as I

pytestmark = pytest.mark.gpu

CAP = 50_000


def say(*a):
    print(*a, flush=True)


def host(t):
    return t.detach().cpu().numpy()


def ra_of(p):
    return S.RaOpts(coarse_stride=p.coarse_stride, coarse_n=p.coarse_n, C=p.ra_C, M=p.ra_M,
                    q=p.ra_q, tol=p.ra_tol)


def test_kruzkov_global_fp64_bit_exact():
    p = W.kruzkov_problem(n=97)
    say("case: kruzkov global fp64 97")
    V, _, st = S.solve(S.to_device(p, torch.float64), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, _, _ = O.solve(p)
    assert st["converged"]
    assert np.array_equal(host(V), Vo)


def test_kruzkov_global_fp32():
    p = W.kruzkov_problem(n=129)
    V, _, st = S.solve(S.to_device(p, torch.float32), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, _, _ = O.solve(p)
    err = np.abs(host(V).astype(np.float64) - Vo).max()
    say("  kruzkov fp32 sup err", err)
    assert st["converged"] and err <= 1e-5


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_kruzkov_isa(dtype):
    p = W.kruzkov_problem(n=129)
    dp = S.to_device(p, dtype)
    V, owner, member, label, _, Vs, st = S.isa(dp, ra_of(p), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vbar, own_o, rec, Vs_o, _ = I.isa(p)
    assert st["converged"]
    assert np.array_equal(host(member), rec.member)
    assert np.array_equal(host(label), rec.label)
    if dtype == torch.float64:
        assert np.array_equal(host(V), Vbar)
    else:
        err = np.abs(host(V).astype(np.float64) - Vbar).max()
        say("  kruzkov isa fp32 sup err", err)
        assert err <= 1e-5


def test_kruzkov_block_async_equals_jacobi():
    p = W.kruzkov_problem(n=257)
    dp = S.to_device(p, torch.float32)
    ra = ra_of(p)
    member, _, _ = S.reconstruct(dp, ra)
    Vj = S.solve_isa(dp, ra, member, S.SolveOpts(tol=0.0, max_sweeps=CAP), want_sets=True)
    for k in (4, 8):
        Va = S.solve_isa(dp, ra, member, S.SolveOpts(tol=0.0, max_sweeps=CAP, local_iters=k),
                         want_sets=True)
        say("  kruzkov local", k, "launches", Va[-1]["sweeps_max"], "vs", Vj[-1]["sweeps_max"])
        assert torch.equal(Va[3], Vj[3])


def test_full_size_kruzkov_benchmark_configuration():
    """The benchmark's Kruzkov workload (513^2, coarse 65^2) in its launch
    configuration (tuned kernels, 8 local iterations, coarse: 4 local iterations):
    sets and labels bit-exact, and every set's FP32 values a fixed point of the
    oracle's FP64 operator up to FP32 rounding."""
    from tests.test_gpu_drift import _fixed_point_residuals
    p = W.kruzkov_problem()
    dp = S.to_device(p, torch.float32)
    ra = ra_of(p)
    ra.autotune, ra.local_iters = 1, 4
    member, label, _ = S.reconstruct(dp, ra)
    rec = I.reconstruct(p)
    assert np.array_equal(host(member), rec.member)
    assert np.array_equal(host(label), rec.label)
    V, own, pol, Vs, st = S.solve_isa(dp, ra, member,
                                      S.SolveOpts(tol=0.0, max_sweeps=CAP, autotune=1,
                                                  local_iters=8), want_sets=True)
    assert st["converged"]
    r = _fixed_point_residuals(p, member, host(Vs).reshape(p.n_comp, p.N))
    say("  fixed-point residuals", r, "launches", st["sweeps_max"])
    assert max(r) <= 2e-6


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_batched_kruzkov_matches_oracle(dtype):
    """A batch mixing Kruzkov problems of different sizes with a discounted control
    problem: sets and labels bit-exact per problem, FP64 values bit-exact, FP32
    within 1e-5."""
    probs = [W.kruzkov_problem(n=n, m=16, n_disks=k).with_(coarse_n=(nK, nK),
                                                           name=f"kruzkov_batch{n}")
             for n, k, nK in ((49, 2, 17), (65, 4, 21), (33, 1, 11))]
    probs.append(W.c2_multitarget(n=41, m=16).with_(coarse_n=(11, 11), name="discounted"))
    say("case: batched kruzkov", dtype)
    dps = [S.to_device(p, dtype) for p in probs]
    Vs, mem, lab, own, per, tot = S.solve_batched(dps, [ra_of(p) for p in probs],
                                                  S.SolveOpts(tol=0.0, max_sweeps=CAP))
    assert tot["converged"]
    for p, V, m, l in zip(probs, Vs, mem, lab):
        Vbar, owner, rec, _, _ = I.isa(p)
        assert np.array_equal(host(m), rec.member), p.name
        assert np.array_equal(host(l), rec.label), p.name
        Vg = host(V).astype(np.float64)
        if dtype == torch.float64:
            assert np.array_equal(Vg, Vbar), p.name
        else:
            assert np.abs(Vg - Vbar).max() <= 1e-5, p.name
