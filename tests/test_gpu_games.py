"""Differential games (the maximum over the evader's choices b_l of the minimum
over the pursuer's controls a_k, paper Sec. 2-3) and per-axis speed factors on the
GPU against the oracle: FP64 bit-exact, FP32 within 1e-5, sets and labels
bit-exact, block-asynchronous sweeps equal to Jacobi bit for bit."""
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


def pe(n, split=4, **kw):
    return W.pursuit_evasion_problem(n, split=split, m_a=16, m_b=4, **kw)


@pytest.mark.parametrize("case", ["strip_game41", "pe65"])
def test_game_global_fp64_bit_exact(case):
    p = W.strip_game_problem(41) if case == "strip_game41" else pe(65, split=1)
    say("case: game global fp64", case)
    V, _, st = S.solve(S.to_device(p, torch.float64), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, so, _ = O.solve(p)
    say("  sweeps gpu", st["sweeps_max"], "oracle", so)
    assert st["converged"]
    assert np.array_equal(host(V), Vo)


def test_game_global_fp32():
    p = pe(129, split=1)
    say("case: game global fp32 pe129")
    V, _, st = S.solve(S.to_device(p, torch.float32), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, _, _ = O.solve(p)
    err = np.abs(host(V).astype(np.float64) - Vo).max()
    say("  sup err", err, "sweeps", st["sweeps_max"])
    assert st["converged"] and err <= 1e-5


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_game_isa(dtype):
    """Pursuit-evasion, capture ball split in 4 arcs, coarse grid of 25^2 under 97^2
    (not nested): sets and labels bit-exact; FP64 values bit-exact, FP32 within 1e-5."""
    p = pe(97).with_(coarse_n=(25, 25))
    say("case: game isa", dtype)
    dp = S.to_device(p, dtype)
    V, owner, member, label, _, Vs, st = S.isa(dp, ra_of(p), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vbar, own_o, rec, Vs_o, _ = I.isa(p)
    assert st["converged"]
    assert np.array_equal(host(member), rec.member)
    assert np.array_equal(host(label), rec.label)
    if dtype == torch.float64:
        assert np.array_equal(host(V), Vbar)
        assert np.array_equal(host(owner), own_o)
    else:
        err = np.abs(host(V).astype(np.float64) - Vbar).max()
        say("  sup err", err)
        assert err <= 1e-5


def test_game_block_async_equals_jacobi():
    p = pe(129).with_(coarse_n=(33, 33))
    dp = S.to_device(p, torch.float32)
    member, _, _ = S.reconstruct(dp, ra_of(p))
    Vj = S.solve_isa(dp, ra_of(p), member, S.SolveOpts(tol=0.0, max_sweeps=CAP), want_sets=True)
    for k in (2, 8):
        Va = S.solve_isa(dp, ra_of(p), member,
                         S.SolveOpts(tol=0.0, max_sweeps=CAP, local_iters=k), want_sets=True)
        say("  game, local iterations", k, "launches", Va[-1]["sweeps_max"], "vs",
            Vj[-1]["sweeps_max"])
        assert torch.equal(Va[3], Vj[3])


def _game3d(n=17):
    """3D game: pursuer on 16 Fibonacci directions, evader on 3 directions of length
    0.3, per-axis speed factors from seeded smooth fields, 2 balls."""
    p = W.c3_aniso3d(n=n, m=16, n_balls=2, r=0.2)
    X = W.node_coords(p.n, p.lo, p.hi)
    g = W.gaussian_field(tuple(reversed(p.n)), 0.2 / p.dx[0], 808).reshape(-1)
    fac = np.stack([1.0 + 0.2 * g, 0.8 + 0.1 * X[:, 0], 1.1 - 0.1 * X[:, 2]], axis=1)
    vb = 0.3 * np.array([[1.0, 0.0, 0.0], [0.0, -0.6, 0.8], [-0.6, 0.0, -0.8]])
    return p.with_(speed=W.f32(fac), velocity_b=vb, v_ghost=2.0)


def test_game_3d_fp64_bit_exact():
    p = _game3d()
    say("case: game 3d fp64")
    V, _, st = S.solve(S.to_device(p, torch.float64), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, _, _ = O.solve(p)
    assert st["converged"]
    assert np.array_equal(host(V), Vo)


def test_game_3d_block_async_fp32():
    p = _game3d(21)
    dp = S.to_device(p, torch.float32)
    Vj, _, sj = S.solve(dp, S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Va, _, sa = S.solve(dp, S.SolveOpts(tol=0.0, max_sweeps=CAP, local_iters=4))
    Vo, _, _, _ = O.solve(p)
    err = np.abs(host(Vj).astype(np.float64) - Vo).max()
    say("  3d game fp32 sup err", err, "launches", sa["sweeps_max"], "vs", sj["sweeps_max"])
    assert err <= 1e-5
    assert torch.equal(Va, Vj)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_axis_speed_control_problem(dtype):
    """A control problem whose speed has one factor per axis (the multitarget field
    on x1, a smooth ramp on x2)."""
    base = W.c2_multitarget(n=129, m=32)
    X = W.node_coords(base.n, base.lo, base.hi)
    fac = np.stack([np.asarray(base.speed), 0.6 + 0.3 * (X[:, 0] + 1.0)], axis=1)
    p = base.with_(speed=W.f32(fac))
    V, _, st = S.solve(S.to_device(p, dtype), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, _, _ = O.solve(p)
    assert st["converged"]
    if dtype == torch.float64:
        assert np.array_equal(host(V), Vo)
    else:
        assert np.abs(host(V).astype(np.float64) - Vo).max() <= 1e-5


def test_game_autotune_and_policy_rejection():
    """The autotuner's game candidates give each tile one thread group, and the
    result matches the default configuration's (FP32 feet are tile-local, so another
    tile shape changes the last bits); a policy output is refused."""
    p = pe(97, split=1)
    dp = S.to_device(p, torch.float32)
    V0, _, s0 = S.solve(dp, S.SolveOpts(tol=0.0, max_sweeps=CAP))
    V1, _, s1 = S.solve(dp, S.SolveOpts(tol=0.0, max_sweeps=CAP, autotune=1))
    say("  autotuned variant", s1["variant"], "mode", s1["mode"])
    assert s1["variant"] not in (13, 14, 15)          # the split-control variants
    assert float((V0 - V1).abs().max()) <= 1e-6
    with pytest.raises(S.SlError) as e:
        S.solve(dp, S.SolveOpts(tol=0.0, max_sweeps=CAP, want_policy=True))
    assert e.value.status == -3


def test_full_size_pursuit_evasion_benchmark_configuration():
    """The benchmark's game workload (513^2, 32 x 9 controls, 4 arcs, coarse 65^2)
    in the launch configuration it times (tuned kernels, 4 local iterations): sets
    and labels bit-exact against the oracle's reconstruction, and every set's FP32
    values a fixed point of the oracle's FP64 game operator up to FP32 rounding."""
    from tests.test_gpu_drift import _fixed_point_residuals
    p = W.pursuit_evasion_problem(513, split=4, m_a=32, m_b=8).with_(coarse_stride=8)
    say("case: full-size pursuit-evasion 513")
    dp = S.to_device(p, torch.float32)
    ra = ra_of(p)
    ra.autotune, ra.local_iters = 1, 4
    member, label, _ = S.reconstruct(dp, ra)
    rec = I.reconstruct(p)
    assert np.array_equal(host(member), rec.member)
    assert np.array_equal(host(label), rec.label)
    V, own, pol, Vs, st = S.solve_isa(dp, ra, member,
                                      S.SolveOpts(tol=0.0, max_sweeps=CAP, autotune=1,
                                                  local_iters=4), want_sets=True)
    assert st["converged"]
    r = _fixed_point_residuals(p, member, host(Vs).reshape(p.n_comp, p.N))
    say("  fixed-point residuals", r, "launches", st["sweeps_max"])
    assert max(r) <= 2e-6


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_batched_games_match_oracle(dtype):
    """A batch of games of different sizes and splits (the pursuit-evasion controls
    and cost with a scalar speed field, which the batch takes; per-axis factors it
    does not), solved in one batched call: sets and labels bit-exact per problem,
    FP64 values bit-exact, FP32 within 1e-5."""
    probs = []
    for k, (n, split, nK) in enumerate([(33, 1, 9), (49, 4, 13), (41, 4, 21), (57, 1, 15)]):
        X = W.node_coords((n, n), (-1.0, -1.0), (1.0, 1.0))
        probs.append(W.pursuit_evasion_problem(n, split=split, m_a=12, m_b=4)
                     .with_(speed=W.f32(1.0 + 0.3 * X[:, 1] ** 2), coarse_n=(nK, nK),
                            name=f"game_batch{k}"))
    say("case: batched games", dtype, [p.n[0] for p in probs])
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


def test_batched_games_with_axis_factors_match_oracle():
    """Pursuit-evasion games with their per-axis speed factors (x2 + 1, 1), mixed
    with a control problem, in one FP64 batch: bit-exact per problem."""
    probs = [W.pursuit_evasion_problem(n, split=s, m_a=12, m_b=4).with_(coarse_n=(nK, nK),
                                                                         name=f"pe_axes{k}")
             for k, (n, s, nK) in enumerate([(33, 4, 9), (49, 1, 13)])]
    X = W.node_coords((41, 41), (-1.0, -1.0), (1.0, 1.0))
    ctrl = W.c2_multitarget(n=41, m=16)
    probs.append(ctrl.with_(speed=W.f32(np.stack([np.asarray(ctrl.speed),
                                                  1.0 + 0.1 * X[:, 0]], axis=1)),
                            velocity_b=None, coarse_n=(11, 11), name="axes_control"))
    dps = [S.to_device(p, torch.float64) for p in probs]
    Vs, mem, lab, own, per, tot = S.solve_batched(dps, [ra_of(p) for p in probs],
                                                  S.SolveOpts(tol=0.0, max_sweeps=CAP))
    assert tot["converged"]
    for p, V, m, l in zip(probs, Vs, mem, lab):
        Vbar, owner, rec, _, _ = I.isa(p)
        assert np.array_equal(host(m), rec.member), p.name
        assert np.array_equal(host(l), rec.label), p.name
        assert np.array_equal(host(V), Vbar), p.name
