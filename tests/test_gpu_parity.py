"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Bars: FP64 values and every integer output (sets, labels) bit-exact; FP32 values
within 1e-5 in the sup norm of the oracle's FP64 fixed point, both iterated until
nothing changes; policies equal wherever the oracle's best-to-second gap exceeds
the FP32 error."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1405_3521_amd as S
import workloads as W
from oracle import isa as I

pytestmark = pytest.mark.gpu

# sweep cap of the fixed-point solves: a solve that has not converged by then
# returns (and fails its checks) instead of running on
CAP = 50_000

DEV = "cuda:0"


def ra_of(p):
    return S.RaOpts(coarse_stride=p.coarse_stride, coarse_n=p.coarse_n, C=p.ra_C, M=p.ra_M, q=p.ra_q, tol=p.ra_tol)


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)


# ----------------------------------------------------------------- global solves
@pytest.mark.parametrize("n", [101, 67])
def test_global_fp64_bit_exact(n):
    """FP64 global solve: same operation order as the oracle -> identical bits."""
    p = W.c1_eikonal(n)
    say("case: global fp64 eikonal", n)
    V, _, st = S.solve(S.to_device(p, torch.float64), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, so, _ = O.solve(p)
    Vg = host(V)
    assert np.array_equal(Vg, Vo), np.abs(Vg - Vo).max()
    assert st["sweeps_max"] == so
    assert st["converged"]


def test_global_fp64_c1_tolerance_stop():
    """C1 configuration: stop at sup-change < 1e-10; same sweep count and iterate."""
    p = W.c1_eikonal(101)
    V, _, st = S.solve(S.to_device(p, torch.float64), S.SolveOpts(tol=1e-10))
    Vo, _, so, ro = O.solve(p, tol=1e-10)
    assert st["sweeps_max"] == so
    assert np.array_equal(host(V), Vo)
    assert st["residual"] == ro


@pytest.mark.parametrize("n,m", [(129, 64), (97, 32), (130, 16)])
def test_global_fp32_parity(n, m):
    """FP32 global solve vs FP64 oracle, both to stagnation: sup <= 1e-5."""
    if (n - 1) % 2:
        p = W.c2_multitarget(n=n, m=m).with_(coarse_stride=1)
    else:
        p = W.c2_multitarget(n=n, m=m)
    say("case: global fp32 multitarget", n, m)
    V, pol, st = S.solve(S.to_device(p, torch.float32), S.SolveOpts(tol=0.0, max_sweeps=CAP, want_policy=True))
    Vo, polo, _, _ = O.solve(p)
    err = np.abs(host(V).astype(np.float64) - Vo).max()
    say("  sup err", err, "sweeps", st["sweeps_max"])
    assert err <= 1e-5
    # policy: equal where the oracle's decision is clear
    TV, _ = O.apply_T(p, Vo)
    pg = host(pol).astype(np.int64)
    free = polo >= 0
    assert (pg[~free] == 255).all()
    gaps = _gaps(p, Vo)
    clear = free & (gaps > 1e-4)
    assert (pg[clear] == polo[clear]).mean() == 1.0


def _gaps(p, V):
    """Best-to-second candidate gap per node (oracle, FP64), by evaluating T with
    each control removed in turn is too slow; use the control-restricted apply."""
    best = None
    vals = []
    for k in range(p.m):
        q = p.with_(velocity=p.velocity[k:k + 1])
        TV, _ = O.apply_T(q, V)
        vals.append(TV)
    A = np.sort(np.stack(vals), axis=0)
    return A[1] - A[0]


def test_single_sweep_fp64_equals_oracle():
    """max_sweeps = 1 -> SL_NOT_CONVERGED, V = T(V0) bit for bit."""
    p = W.c2_multitarget(n=65, m=32)
    V, _, st = S.solve(S.to_device(p, torch.float64), S.SolveOpts(tol=0.0, max_sweeps=1))
    assert not st["converged"]
    Vo, _, _, _ = O.solve(p, max_sweeps=1)
    assert np.array_equal(host(V), Vo)


# -------------------------------------------------------------- reconstruction
@pytest.mark.parametrize("n", [129, 257])
def test_reconstruction_bit_exact(n):
    """RA on the coarse grid (FP64, fixed operation order) + Con projection: the
    sets and labels equal the oracle's bit for bit, on K and on the fine grid."""
    p = W.c2_multitarget(n=n, m=64)
    say("case: reconstruct", n, "stride", p.coarse_stride)
    dp = S.to_device(p, torch.float32)
    member, label, st, mK, lK = S.reconstruct(dp, ra_of(p), want_coarse=True)
    rec = I.reconstruct(p)
    assert np.array_equal(host(mK), rec.member_K)
    assert np.array_equal(host(lK), rec.label_K)
    assert np.array_equal(host(member), rec.member)
    assert np.array_equal(host(label), rec.label)


@pytest.mark.parametrize("local", [0, 8])
def test_reconstruction_full_size_c2_labels(local):
    """Full C2 size (1025^2, coarse 129^2): labels and sets bit-exact, with Jacobi
    coarse sweeps and with the benchmark's coarse configuration (tuned kernels,
    8 local iterations per tile and launch, tol 0)."""
    p = W.c2_multitarget()
    say("case: reconstruct full c2, coarse local iterations", local)
    dp = S.to_device(p, torch.float32)
    ra = ra_of(p)
    ra.local_iters = local
    ra.autotune = 1 if local else 0
    member, label, st, mK, lK = S.reconstruct(dp, ra, want_coarse=True)
    probK = I.coarse_problem(p)
    mKo, lKo, _, _, _, _ = I.reconstruct_on(probK)
    assert np.array_equal(host(mK), mKo)
    assert np.array_equal(host(lK), lKo)
    mem, lab = I.project(mKo, lKo, probK.n, p.n)
    assert np.array_equal(host(member), mem)
    assert np.array_equal(host(label), lab)


@pytest.mark.parametrize("n,nK", [(129, (47, 53)), (257, (61, 61)), (100, (41, 41))])
def test_reconstruction_bit_exact_non_nested_coarse_grid(n, nK):
    """A coarse grid of any node counts (not nested in the fine grid): Q1 coarse
    data, nearest-node targets, Con(.) located in integers; sets and labels equal
    the oracle's bit for bit, on K and on the fine grid."""
    p = W.c2_multitarget(n=n, m=64).with_(coarse_n=nK)
    say("case: reconstruct non-nested", n, nK)
    dp = S.to_device(p, torch.float32)
    member, label, st, mK, lK = S.reconstruct(dp, ra_of(p), want_coarse=True)
    rec = I.reconstruct(p)
    assert np.array_equal(host(mK), rec.member_K)
    assert np.array_equal(host(lK), rec.label_K)
    assert np.array_equal(host(member), rec.member)
    assert np.array_equal(host(label), rec.label)


def test_isa_fp64_bit_exact_non_nested_with_cost():
    """FP64 ISA with a running cost, exit costs g and a 35^2 coarse grid under a
    97^2 fine grid: every value and owner bit-exact."""
    p = W.c2_multitarget(n=97, m=32)
    rng = np.random.Generator(np.random.PCG64(31))
    p = p.with_(cost=W.f32(np.exp(rng.normal(0, 0.3, p.N))), v_ghost=4.0,
                g=W.f32(rng.uniform(0, 0.2, p.N)), coarse_n=(35, 35))
    say("case: isa fp64 non-nested cost")
    dp = S.to_device(p, torch.float64)
    V, owner, member, label, _, Vs, st = S.isa(dp, ra_of(p), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vbar, own_o, rec, Vs_o, _ = I.isa(p)
    assert np.array_equal(host(member), rec.member)
    assert np.array_equal(host(V), Vbar)
    assert np.array_equal(host(owner), own_o)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_isa_single_call_equals_two_calls(dtype):
    """sl_isa (one call) against sl_reconstruct followed by sl_solve_isa: the same
    kernels on the same data, so sets, labels, values, owners and per-set values
    are equal bit for bit (Jacobi sweeps; FP64 also equals the oracle)."""
    p = W.c2_multitarget(n=97, m=32)
    say("case: isa single call vs two calls", dtype)
    dp = S.to_device(p, dtype)
    ra = ra_of(p)
    opts = S.SolveOpts(tol=0.0, max_sweeps=CAP)
    V, owner, member, label, _, Vs, st = S.isa(dp, ra, opts, want_sets=True)
    m2, l2, st_ra = S.reconstruct(dp, ra)
    V2, o2, _, Vs2, st2 = S.solve_isa(dp, ra, m2, opts, want_sets=True)
    assert st["converged"] and st2["converged"]
    for a, b in ((member, m2), (label, l2), (V, V2), (owner, o2), (Vs, Vs2)):
        assert np.array_equal(host(a), host(b))
    assert st["sweeps_max"] == st2["sweeps_max"]
    assert st["ra_sweeps_max"] == st_ra["ra_sweeps_max"]
    assert st["ms_ra"] > 0.0 and st["ms_total"] >= st["ms_ra"]
    if dtype == torch.float64:
        Vbar, _, rec, _, _ = I.isa(p)
        assert np.array_equal(host(member), rec.member)
        assert np.array_equal(host(label), rec.label)
        assert np.array_equal(host(V), Vbar)


def test_prepared_isa_solver_equals_isa():
    """IsaSolver (arguments marshalled once, outputs kept) gives what isa gives,
    call after call; FP64 equals the oracle bit for bit."""
    p = W.c2_multitarget(n=97, m=32)
    say("case: prepared isa solver")
    dp = S.to_device(p, torch.float64)
    ra = ra_of(p)
    opts = S.SolveOpts(tol=0.0, max_sweeps=CAP)
    solver = S.IsaSolver(dp, ra, want_sets=True)
    ref = S.isa(dp, ra, opts, want_sets=True)
    Vbar, own_o, rec, _, _ = I.isa(p)
    for _ in range(2):
        V, owner, member, label, _, Vs, st = solver.solve(opts)
        assert st["converged"]
        for a, b in ((V, ref[0]), (owner, ref[1]), (member, ref[2]), (label, ref[3]), (Vs, ref[5])):
            assert np.array_equal(host(a), host(b))
        assert np.array_equal(host(V), Vbar)
        assert np.array_equal(host(member), rec.member)


def test_full_size_c2_every_configuration():
    """The benchmark's problem (1025^2, 64 controls, 4 disks), every sweep
    configuration of the autotuner: candidates of one tile shape give the same
    FP32 values bit for bit (neither the schedule nor the split of the controls
    over thread groups changes the arithmetic), all agree within 1e-5, and the
    result is a fixed point of the oracle's FP64 operator on every set up to FP32
    rounding (a check that needs one oracle sweep, not a whole solve)."""
    p = W.c2_multitarget()
    say("case: full-size c2, every configuration")
    dp = S.to_device(p, torch.float32)
    ra = ra_of(p)
    member, label, _ = S.reconstruct(dp, ra)
    nc = S.lib().sl_tune_candidates(2, 0)
    by_tile, ref = {}, None
    for k in range(1, nc + 1):
        V, own, pol, Vs, st = S.solve_isa(dp, ra, member,
                                          S.SolveOpts(tol=0.0, max_sweeps=CAP, autotune=-k),
                                          want_sets=True)
        assert st["converged"], k
        Vh = host(Vs).reshape(p.n_comp, p.N)
        say("  candidate", k, "tile", st["tile"], "mode", st["mode"], "sweeps", st["sweeps_max"])
        key = tuple(st["tile"])
        if key in by_tile:
            assert np.array_equal(Vh, by_tile[key]), k
        else:
            by_tile[key] = Vh
        if ref is None:
            ref = Vh
        else:
            assert np.abs(Vh.astype(np.float64) - ref).max() <= 1e-5, k
    mem = host(member)
    fixed = O.fixed_mask(p)
    for i in range(p.n_comp):
        dom = ((mem >> i) & 1).astype(np.uint8)
        Vi = ref[i].astype(np.float64)
        TV, _ = O.apply_T(p, Vi, fixed=fixed, dom=dom)
        on = dom.astype(bool) & (np.asarray(p.target) < 0)
        r = np.abs(TV[on] - Vi[on]).max()
        say("  set", i, "fixed-point residual", r)
        assert r <= 2e-6


# ------------------------------------------------------------------------- ISA
@pytest.mark.parametrize("n", [129, 257])
def test_isa_fp32_parity(n):
    """Whole ISA in FP32 vs the oracle's FP64 ISA: sup <= 1e-5 on the assembled
    value and on every set's value; owner equal where the sets' values differ
    clearly."""
    p = W.c2_multitarget(n=n, m=64)
    say("case: isa fp32", n)
    dp = S.to_device(p, torch.float32)
    V, owner, member, label, _, Vs, st = S.isa(dp, ra_of(p), S.SolveOpts(tol=0.0, max_sweeps=CAP),
                                               want_sets=True)
    Vbar, own_o, rec, Vs_o, _ = I.isa(p)
    assert st["converged"]
    assert np.array_equal(host(member), rec.member)
    err = np.abs(host(V).astype(np.float64) - Vbar).max()
    say("  sup err", err, "sweeps", st["sweeps_max"])
    assert err <= 1e-5
    Vsg = host(Vs).reshape(p.n_comp, p.N).astype(np.float64)
    for i in range(p.n_comp):
        on = ((rec.member >> i) & 1).astype(bool)
        assert np.abs(Vsg[i][on] - Vs_o[i][on]).max() <= 1e-5
    # owner: compare where the best and second-best set differ by > 1e-4
    stack = np.where(((rec.member[None, :] >> np.arange(p.n_comp)[:, None]) & 1).astype(bool),
                     np.stack(Vs_o), np.inf)
    srt = np.sort(stack, axis=0)
    clear = (srt[1] - srt[0]) > 1e-4
    assert (host(owner)[clear] == own_o[clear]).all()


def test_isa_fp64_bit_exact():
    """FP64 ISA: every set's solve and the assembly are bit-exact."""
    p = W.c2_multitarget(n=97, m=32)
    dp = S.to_device(p, torch.float64)
    V, owner, member, label, _, Vs, st = S.isa(dp, ra_of(p), S.SolveOpts(tol=0.0, max_sweeps=CAP),
                                               want_sets=True)
    Vbar, own_o, rec, Vs_o, _ = I.isa(p)
    assert np.array_equal(host(V), Vbar)
    assert np.array_equal(host(owner), own_o)


# --------------------------------------------------------------------------- 3D
def test_global_3d_fp64_bit_exact():
    p = W.c3_aniso3d(n=21, m=32, n_balls=3, r=0.15)
    say("case: 3d fp64 global")
    V, _, st = S.solve(S.to_device(p, torch.float64), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, so, _ = O.solve(p)
    assert np.array_equal(host(V), Vo)


@pytest.mark.parametrize("n,nK", [(33, None), (41, None), (30, (11, 13, 9))])
def test_isa_3d_fp32_parity(n, nK):
    p = W.c3_aniso3d(n=n, m=64, n_balls=4, r=0.12)
    if nK is not None:
        p = p.with_(coarse_n=nK)
    say("case: 3d fp32 isa", n, "stride", p.coarse_stride, "coarse nodes", nK)
    dp = S.to_device(p, torch.float32)
    V, owner, member, label, _, Vs, st = S.isa(dp, ra_of(p), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vbar, own_o, rec, Vs_o, _ = I.isa(p)
    assert st["converged"]
    assert np.array_equal(host(member), rec.member)
    assert np.array_equal(host(label), rec.label)
    err = np.abs(host(V).astype(np.float64) - Vbar).max()
    say("  sup err", err, "sweeps", st["sweeps_max"])
    assert err <= 1e-5


# ------------------------------------------------------------------- edge cases
def test_no_target_is_an_error():
    p = W.c1_eikonal(33)
    p = p.with_(target=np.full(p.N, -1, dtype=np.int8))
    with pytest.raises(S.SlError) as e:
        S.solve(S.to_device(p, torch.float32))
    assert e.value.status == -2


def test_nan_speed_is_an_error():
    p = W.c2_multitarget(n=33, m=16)
    sp = p.speed.copy()
    sp[5] = np.nan
    with pytest.raises(S.SlError) as e:
        S.solve(S.to_device(p.with_(speed=sp), torch.float32))
    assert e.value.status == -1


def test_tiny_grid_and_whole_target():
    """3x3 grid; and a grid whose every node is a target (nothing to solve)."""
    p = W.c1_eikonal(3)
    V, _, st = S.solve(S.to_device(p, torch.float64))
    Vo, _, _, _ = O.solve(p)
    assert np.array_equal(host(V), Vo)
    q = p.with_(target=np.zeros(p.N, dtype=np.int8))
    V, _, st = S.solve(S.to_device(q, torch.float64))
    assert (host(V) == 0).all()


# ------------------------------------------------------ every kernel configuration
@pytest.mark.parametrize("dim", [2, 3])
def test_every_tuner_candidate_matches_oracle(dim):
    """Each (tile shape, work schedule) the autotuner may pick gives the oracle's
    fixed point (FP32 <= 1e-5; FP64 bit-exact), with tile skipping active."""
    if dim == 2:
        p = W.c2_multitarget(n=97, m=32)
    else:
        p = W.c3_aniso3d(n=25, m=32, n_balls=3, r=0.15)
    Vo, _, _, _ = O.solve(p)
    for dtype in (torch.float32, torch.float64):
        code = 0 if dtype == torch.float32 else 1
        ncand = S.lib().sl_tune_candidates(dim, code)
        assert ncand >= 3
        dp = S.to_device(p, dtype)
        for k in range(ncand):
            V, _, st = S.solve(dp, S.SolveOpts(tol=0.0, max_sweeps=CAP, autotune=-(k + 1)))
            Vg = host(V).astype(np.float64)
            say("  candidate", dim, dtype, k, st["tile"], st["mode"], np.abs(Vg - Vo).max())
            if dtype == torch.float64:
                assert np.array_equal(Vg, Vo), (k, st["tile"], st["mode"])
            else:
                assert np.abs(Vg - Vo).max() <= 1e-5, (k, st["tile"], st["mode"])


def test_autotuned_isa_matches_oracle():
    p = W.c2_multitarget(n=129, m=64)
    dp = S.to_device(p, torch.float32)
    V, owner, member, label, _, _, st = S.isa(dp, ra_of(p), S.SolveOpts(tol=0.0, max_sweeps=CAP, autotune=2))
    Vbar, _, rec, _, _ = I.isa(p)
    assert np.abs(host(V).astype(np.float64) - Vbar).max() <= 1e-5
    say("  tuned:", st["tile"], st["mode"])


def test_reconstruction_with_tuned_coarse_kernels():
    """The coarse FP64 pass gives the oracle's sets whatever kernel the tuner picks."""
    p = W.c2_multitarget(n=257, m=64)
    dp = S.to_device(p, torch.float32)
    ra = ra_of(p)
    ra.autotune = 2
    member, label, st, mK, lK = S.reconstruct(dp, ra, want_coarse=True)
    rec = I.reconstruct(p)
    assert np.array_equal(host(mK), rec.member_K)
    assert np.array_equal(host(member), rec.member)
    assert np.array_equal(host(label), rec.label)
