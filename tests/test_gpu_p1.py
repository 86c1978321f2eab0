"""P1 interpolation on the Kuhn simplices of each cell (2D and 3D) on the GPU against the
oracle: FP64 bit-exact (the same nested evaluation and an exact division), FP32
within 1e-5, sets and labels bit-exact, block-asynchronous sweeps equal to Jacobi
bit for bit, and the 1025^2 multitarget workload in the benchmark's launch
configuration a fixed point of the oracle's P1 operator."""
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


def p1(n, **kw):
    return W.c2_multitarget(n=n, m=32, **kw).with_(interp="p1")


@pytest.mark.parametrize("li", [0, 8])
def test_p1_global_fp64_bit_exact(li):
    p = p1(97)
    say("case: p1 global fp64 97 local", li)
    V, pol, st = S.solve(S.to_device(p, torch.float64),
                         S.SolveOpts(tol=0.0, max_sweeps=CAP, local_iters=li, want_policy=True))
    Vo, pol_o, _, _ = O.solve(p)
    assert st["converged"]
    assert np.array_equal(host(V), Vo)
    free = pol_o >= 0
    assert np.array_equal(host(pol).astype(np.int64)[free], pol_o[free])


def test_p1_global_fp32():
    p = p1(129)
    say("case: p1 global fp32 129")
    V, _, st = S.solve(S.to_device(p, torch.float32), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, _, _ = O.solve(p)
    err = np.abs(host(V).astype(np.float64) - Vo).max()
    say("  sup err", err)
    assert st["converged"] and err <= 1e-5
    # not the Q1 solution
    Vq, _, _, _ = O.solve(p.with_(interp="q1"))
    assert np.abs(Vq - Vo).max() > 1e-4


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_p1_isa(dtype):
    p = p1(129)
    say("case: p1 isa 129", dtype)
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


def test_p1_block_async_equals_jacobi_and_tuned_configs():
    p = p1(257)
    say("case: p1 block-async 257")
    dp = S.to_device(p, torch.float32)
    ra = ra_of(p)
    member, _, _ = S.reconstruct(dp, ra)
    Vj = S.solve_isa(dp, ra, member, S.SolveOpts(tol=0.0, max_sweeps=CAP), want_sets=True)
    for k in (1, 8):
        Va = S.solve_isa(dp, ra, member, S.SolveOpts(tol=0.0, max_sweeps=CAP, local_iters=k),
                         want_sets=True)
        say("  local", k, "launches", Va[-1]["sweeps_max"], "vs", Vj[-1]["sweeps_max"])
        assert torch.equal(Va[3], Vj[3])
    # every P1 candidate of the tuner (FP32 tile-local coordinates differ in the
    # last bits across tile shapes): within 1e-6 of the default
    Vt = S.solve_isa(dp, ra, member, S.SolveOpts(tol=0.0, max_sweeps=CAP, autotune=1,
                                                 local_iters=8), want_sets=True)
    err = float((Vt[3] - Vj[3]).abs().max())
    say("  tuned", Vt[-1].get("variant"), "err", err)
    assert err <= 1e-6


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_p1_batch_matches_oracle(dtype):
    """A batch of P1 problems of different sizes (the batch's joint work lists
    share one interpolation): sets and labels bit-exact per problem, FP64 values
    bit-exact, FP32 within 1e-5; a batch mixing P1 and Q1 is refused."""
    probs = [W.c2_multitarget(n=n, m=16, n_disks=k).with_(coarse_n=(nK, nK), interp="p1",
                                                          name=f"p1_batch{n}")
             for n, k, nK in ((49, 2, 17), (65, 4, 21), (33, 1, 11))]
    say("case: batched p1", dtype)
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
    q = probs[0].with_(interp="q1")
    with pytest.raises((S.SlError, ValueError)):
        S.solve_batched([dps[0], S.to_device(q, dtype)], [ra_of(probs[0]), ra_of(q)])


def _pol_u8(pol):
    return np.where(pol < 0, 255, pol).astype(np.uint8)


ADJ_CASES = [
    ("2d_fp32", lambda: W.c5_adjoint(n=129, n_obs=1500).with_(interp="p1"), torch.float32, 1e-4),
    ("2d_fp64", lambda: W.c5_adjoint(n=129, n_obs=1500).with_(interp="p1"), torch.float64, 1e-12),
    ("3d_fp64", lambda: p1_3d(25), torch.float64, 1e-12),
    ("3d_fp32", lambda: p1_3d(25), torch.float32, 1e-4),
]


@pytest.mark.parametrize("name,mk,dtype,tol", ADJ_CASES, ids=[c[0] for c in ADJ_CASES])
def test_p1_adjoint_matches_oracle(name, mk, dtype, tol):
    """The adjoint with P1 feet (scatter to the simplex's vertices with their
    barycentric weights) against the oracle's adjoint: relative l2 within 1e-4
    (FP32) or 1e-12 (FP64); local_iters > 0 runs the same Jacobi iteration."""
    p = mk()
    say("case: p1 adjoint", name)
    V, pol, _, _ = O.solve(p)
    gV = np.random.Generator(np.random.PCG64(21)).normal(size=p.N)
    _, dLdl_o, _, _ = O.adjoint(p, pol, gV)
    dp = S.to_device(p, dtype)
    for li in (0, 4):
        dLdl, st = S.adjoint(dp, torch.as_tensor(_pol_u8(pol), device="cuda:0"),
                             torch.as_tensor(gV, dtype=dtype, device="cuda:0"),
                             tol=0.0, local_iters=li)
        got = host(dLdl).astype(np.float64)
        err = float(np.linalg.norm(got - dLdl_o) / np.linalg.norm(dLdl_o))
        say("  local", li, "rel l2", err, "launches", st["sweeps_max"])
        assert st["converged"] and err <= tol


def test_full_size_p1_benchmark_configuration():
    """The 1025^2 multitarget workload (64 controls, coarse 129^2) with P1, in the
    benchmark's launch configuration (tuned kernels, 8 local iterations; coarse 8):
    sets and labels bit-exact, every set's FP32 values a fixed point of the oracle's
    FP64 P1 operator up to FP32 rounding."""
    from tests.test_gpu_drift import _fixed_point_residuals
    p = W.c2_multitarget().with_(interp="p1")
    say("case: p1 full size 1025")
    dp = S.to_device(p, torch.float32)
    ra = ra_of(p)
    ra.autotune, ra.local_iters = 1, 8
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


def p1_3d(n, m=26):
    return W.c3_aniso3d(n=n, m=m, n_balls=2, r=0.2).with_(interp="p1")


@pytest.mark.parametrize("li", [0, 4])
def test_p1_3d_global_fp64_bit_exact(li):
    p = p1_3d(25)
    say("case: p1 3d global fp64 25 local", li)
    V, _, st = S.solve(S.to_device(p, torch.float64),
                       S.SolveOpts(tol=0.0, max_sweeps=CAP, local_iters=li))
    Vo, _, _, _ = O.solve(p)
    assert st["converged"]
    assert np.array_equal(host(V), Vo)


def test_p1_3d_fp32_and_block_async():
    p = p1_3d(33)
    say("case: p1 3d fp32 33")
    dp = S.to_device(p, torch.float32)
    V, _, st = S.solve(dp, S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, _, _ = O.solve(p)
    err = np.abs(host(V).astype(np.float64) - Vo).max()
    say("  sup err", err)
    assert st["converged"] and err <= 1e-5
    assert np.abs(O.solve(p.with_(interp="q1"))[0] - Vo).max() > 1e-4
    Va, _, sta = S.solve(dp, S.SolveOpts(tol=0.0, max_sweeps=CAP, local_iters=4))
    say("  local 4 launches", sta["sweeps_max"], "vs", st["sweeps_max"])
    assert torch.equal(Va, V)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_p1_3d_isa(dtype):
    p = p1_3d(33)
    say("case: p1 3d isa 33", dtype)
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


def test_p1_3d_tuned_configs():
    """Every 3D P1 tuner candidate (forced one by one) is within 1e-5 of the
    oracle, the FP32 parity bar.  Candidates are not compared bit for bit with each
    other: FP32 foot coordinates are tile-local, so they round differently across
    tile shapes (about 1e-6 apart here)."""
    p = p1_3d(33)
    say("case: p1 3d tuner candidates 33")
    dp = S.to_device(p, torch.float32)
    V0, _, _ = S.solve(dp, S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, _, _ = O.solve(p)
    k = 1
    while True:
        try:
            V, _, st = S.solve(dp, S.SolveOpts(tol=0.0, max_sweeps=CAP, autotune=-k, local_iters=4))
        except S.SlError:
            break
        err = float((V - V0).abs().max())
        err_o = np.abs(host(V).astype(np.float64) - Vo).max()
        say("  candidate", k, "tile", st.get("tile"), "vs default", err, "vs oracle", err_o)
        assert st["converged"] and err_o <= 1e-5
        k += 1
    assert k > 9            # 3 variants x 3 schedules


def test_p1_3d_isa_tuned_coarse_pass():
    """The 3D reconstruction with the tuner over the FP64 P1 coarse kernels and
    block-asynchronous coarse sweeps: sets and labels bit-exact (FP64 coordinates
    are global, so every tile shape gives the same values)."""
    p = p1_3d(33)
    say("case: p1 3d tuned coarse 33")
    dp = S.to_device(p, torch.float32)
    ra = ra_of(p)
    ra.autotune, ra.local_iters = 1, 4
    member, label, _ = S.reconstruct(dp, ra)
    rec = I.reconstruct(p)
    assert np.array_equal(host(member), rec.member)
    assert np.array_equal(host(label), rec.label)
