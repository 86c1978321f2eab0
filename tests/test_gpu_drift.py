"""Control-affine dynamics with a drift, f = drift(x) + c(x) b_k (the Van der Pol
example of Sec. 4.1), on the GPU against the oracle: FP64 bit-exact, FP32 within
1e-5, sets and labels bit-exact."""
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


def _const_drift(n):
    p = W.strip_problem(n, 1.0)
    tid = np.full(p.N, -1, dtype=np.int8)
    tid.reshape(n, n)[:, -1] = 0
    drift = np.zeros((p.N, 2))
    drift[:, 0] = 1.0
    return p.with_(target=tid, n_comp=1, drift=drift, h=(2.0 / (n - 1)) / 2, v_ghost=1.0)


@pytest.mark.parametrize("case", ["vdp65", "const_drift81"])
def test_drift_global_fp64_bit_exact(case):
    p = W.vdp_problem(65, split=1) if case == "vdp65" else _const_drift(81)
    say("case: drift global fp64", case)
    V, _, st = S.solve(S.to_device(p, torch.float64), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, so, _ = O.solve(p)
    assert st["converged"]
    assert np.array_equal(host(V), Vo)


def test_drift_global_fp32():
    p = W.vdp_problem(129, split=1)
    say("case: drift global fp32 vdp129")
    V, _, st = S.solve(S.to_device(p, torch.float32), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, _, _ = O.solve(p)
    err = np.abs(host(V).astype(np.float64) - Vo).max()
    say("  sup err", err, "sweeps", st["sweeps_max"])
    assert st["converged"] and err <= 1e-5


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_drift_isa(dtype):
    """4-way split of the target disk, coarse grid of 25^2 under 97^2: sets and
    labels bit-exact; FP64 values bit-exact, FP32 within 1e-5."""
    p = W.vdp_problem(97, split=4).with_(coarse_n=(25, 25))
    say("case: drift isa", dtype)
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
        say("  sup err", err)
        assert err <= 1e-5


def test_drift_block_async_equals_jacobi():
    p = W.vdp_problem(129, split=4).with_(coarse_n=(33, 33))
    dp = S.to_device(p, torch.float32)
    member, _, _ = S.reconstruct(dp, ra_of(p))
    Vj = S.solve_isa(dp, ra_of(p), member, S.SolveOpts(tol=0.0, max_sweeps=CAP), want_sets=True)
    for k in (2, 8):
        Va = S.solve_isa(dp, ra_of(p), member,
                         S.SolveOpts(tol=0.0, max_sweeps=CAP, local_iters=k), want_sets=True)
        say("  drift, local iterations", k, "launches", Va[-1]["sweeps_max"], "vs",
            Vj[-1]["sweeps_max"])
        assert torch.equal(Va[3], Vj[3])


def test_drift_3d_fp64_bit_exact():
    """3D with a smooth random drift field (a rotation about the z axis plus a
    seeded Gaussian field), FP64 global solve bit-exact."""
    p = W.c3_aniso3d(n=21, m=32, n_balls=3, r=0.15)
    X = W.node_coords(p.n, p.lo, p.hi)
    g = W.gaussian_field(tuple(reversed(p.n)), 0.2 / p.dx[0], 707).reshape(-1)
    drift = np.stack([-0.5 * X[:, 1] + 0.2 * g, 0.5 * X[:, 0], 0.1 * g], axis=1)
    p = p.with_(drift=W.f32(drift))
    V, _, st = S.solve(S.to_device(p, torch.float64), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, _, _ = O.solve(p)
    assert st["converged"]
    assert np.array_equal(host(V), Vo)


def _fixed_point_residuals(p, member, Vs):
    """Largest |T(V_i) - V_i| of the oracle's FP64 operator over each set's free
    nodes (one oracle sweep per set)."""
    mem = host(member)
    fixed = O.fixed_mask(p)
    out = []
    for i in range(p.n_comp):
        dom = ((mem >> i) & 1).astype(np.uint8)
        Vi = Vs[i].astype(np.float64)
        TV, _ = O.apply_T(p, Vi, fixed=fixed, dom=dom)
        on = dom.astype(bool) & (np.asarray(p.target) < 0)
        out.append(float(np.abs(TV[on] - Vi[on]).max(initial=0.0)))
    return out


def test_full_size_vdp_benchmark_configuration():
    """The benchmark's Van der Pol workload (1025^2, 4 slices, coarse 129^2) in the
    launch configuration it times (tuned kernels, 8 local iterations): sets and
    labels bit-exact against the oracle's reconstruction, and every set's FP32
    values a fixed point of the oracle's FP64 operator up to FP32 rounding."""
    p = W.vdp_problem(1025, split=4).with_(coarse_stride=8)
    say("case: full-size vdp 1025")
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
def test_batched_drift_matches_oracle(dtype):
    """A batch of Van der Pol problems of different sizes and splits (drift) in one
    batched call: sets and labels bit-exact per problem, FP64 values bit-exact,
    FP32 within 1e-5."""
    probs = [W.vdp_problem(n, split=s).with_(coarse_n=(nK, nK), name=f"vdp_batch{k}")
             for k, (n, s, nK) in enumerate([(41, 4, 11), (57, 2, 15), (33, 1, 9), (65, 4, 17)])]
    say("case: batched drift", dtype, [p.n[0] for p in probs])
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
