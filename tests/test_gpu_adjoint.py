"""GPU adjoint and autograd against the FP64 oracle.

The adjoint kernel is fed the oracle's inputs (policy, sets, owner, dL/dV) and
must reproduce the oracle's dL/dl (FP32: relative l2 <= 1e-4; FP64: <= 1e-12; the
atomics only change the summation order).  End to end, the autograd gradient of
sum (V[obs] - V_obs)^2 with respect to theta (l = exp(theta)) is checked against
central differences of the oracle's FP64 forward solve."""
import math

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


def say(*a):
    print(*a, flush=True)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def pol_u8(pol):
    return np.where(pol < 0, 255, pol).astype(np.uint8)


def gpu_tol(g, dtype):
    """Atomics change the summation order between iterations, so the adjoint
    state settles only to within a few ulps; the library's stopping test adds a
    rounding allowance, so no extra tolerance is needed."""
    return 0.0


def _obs_grad(p, V, Vobs, obs):
    g = np.zeros(p.N)
    g[obs] = 2.0 * (V[obs] - Vobs)
    return g


LOCAL = [0, 4]        # Jacobi iteration, block-asynchronous tiles


@pytest.mark.parametrize("li", LOCAL)
@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4), (torch.float64, 1e-12)])
@pytest.mark.parametrize("n", [65, 129])
def test_adjoint_kernel_global(n, dtype, tol, li):
    p = W.c5_adjoint(n=n, n_obs=min(2000, n * n // 8))
    say("case: adjoint global", n, dtype)
    V, pol, _, _ = O.solve(p)
    Vt, _, _, _ = O.solve(p.with_(cost=np.exp(p.meta["theta_true"])))
    obs = p.meta["obs"]
    gV = _obs_grad(p, V, Vt[obs], obs)
    _, dLdl_o, it_o, _ = O.adjoint(p, pol, gV)
    dp = S.to_device(p, dtype)
    g_t = torch.as_tensor(gV, dtype=dtype, device=DEV)
    pol_t = torch.as_tensor(pol_u8(pol), device=DEV)
    dLdl, st = S.adjoint(dp, pol_t, g_t, tol=gpu_tol(gV, dtype), local_iters=li)
    err = rel_l2(dLdl.cpu().numpy().astype(np.float64), dLdl_o)
    say("  local", li, "rel l2", err, "launches gpu", st["sweeps_max"], "oracle iters", it_o)
    assert st["converged"]
    assert err <= tol


@pytest.mark.parametrize("li", LOCAL)
def test_adjoint_kernel_isa(li):
    """Sets frozen, dL/dV routed to the owner set, per-set adjoints summed."""
    p = W.c5_adjoint(n=129, n_obs=1500)
    Vbar, owner, rec, Vs, _ = I.isa(p)
    _, pols, _ = I.solve_subdomains(p, rec.member, want_policy=True)
    Vt = I.isa(p.with_(cost=np.exp(p.meta["theta_true"])))[0]
    obs = p.meta["obs"]
    gV = _obs_grad(p, Vbar, Vt[obs], obs)
    dLdl_o, _ = I.adjoint_isa(p, rec.member, pols, owner, gV)
    dp = S.to_device(p, torch.float32)
    pol_t = torch.as_tensor(np.concatenate([pol_u8(q) for q in pols]), device=DEV)
    dLdl, st = S.adjoint(dp, pol_t, torch.as_tensor(gV, dtype=torch.float32, device=DEV),
                         member=torch.as_tensor(rec.member, device=DEV),
                         owner=torch.as_tensor(owner, device=DEV),
                         tol=gpu_tol(gV, torch.float32), local_iters=li)
    err = rel_l2(dLdl.cpu().numpy().astype(np.float64), dLdl_o)
    say("  isa adjoint, local", li, "rel l2", err, "launches", st["sweeps_max"])
    assert err <= 1e-4


@pytest.mark.parametrize("li", LOCAL)
def test_adjoint_full_size_c5(li):
    """Full adjoint configuration (513^2, 2000 observations, 4 targets)."""
    p = W.c5_adjoint()
    say("case: adjoint 513 full size")
    V, pol, _, _ = O.solve(p)
    Vt, _, _, _ = O.solve(p.with_(cost=np.exp(p.meta["theta_true"])))
    obs = p.meta["obs"]
    gV = _obs_grad(p, V, Vt[obs], obs)
    _, dLdl_o, _, _ = O.adjoint(p, pol, gV)
    dp = S.to_device(p, torch.float32)
    dLdl, st = S.adjoint(dp, torch.as_tensor(pol_u8(pol), device=DEV),
                         torch.as_tensor(gV, dtype=torch.float32, device=DEV),
                         tol=gpu_tol(gV, torch.float32), local_iters=li)
    err = rel_l2(dLdl.cpu().numpy().astype(np.float64), dLdl_o)
    say("  local", li, "rel l2", err, "launches", st["sweeps_max"])
    assert err <= 1e-4


@pytest.mark.parametrize("li", LOCAL)
def test_adjoint_nonnegative_for_nonnegative_g(li):
    p = W.c5_adjoint(n=65)
    V, pol, _, _ = O.solve(p)
    rng = np.random.Generator(np.random.PCG64(9))
    gV = rng.random(p.N)
    dp = S.to_device(p, torch.float32)
    dLdl, _ = S.adjoint(dp, torch.as_tensor(pol_u8(pol), device=DEV),
                        torch.as_tensor(gV, dtype=torch.float32, device=DEV),
                        tol=gpu_tol(gV, torch.float32), local_iters=li)
    assert float(dLdl.min()) >= 0.0


@pytest.mark.parametrize("interp", ["q1", "p1"])
@pytest.mark.parametrize("li", LOCAL)
@pytest.mark.parametrize("mode", ["global", "isa"])
def test_autograd_gradient_against_fd(mode, li, interp):
    """theta -> l = exp(theta) -> V (GPU, FP32) -> loss; theta.grad against central
    differences of the oracle's FP64 loss (eps = 1e-6 along dense directions), with
    Q1 and with P1 interpolation (the adjoint then sums over the feet's Kuhn
    simplices)."""
    p = W.c5_adjoint(n=65, n_obs=300)
    if interp == "p1":
        p = p.with_(interp="p1")
    obs = p.meta["obs"]
    member = None
    if mode == "isa":
        rec = I.reconstruct(p)
        member = rec.member

    def oracle_V(theta):
        q = p.with_(cost=np.exp(theta))
        if member is None:
            return O.solve(q)[0]
        Vs, _ = I.solve_subdomains(q, member)
        return I.assemble(Vs, member, q.v_ghost)[0]

    Vobs = oracle_V(p.meta["theta_true"])[obs]

    def loss_o(theta):
        return float(np.sum((oracle_V(theta)[obs] - Vobs) ** 2))

    dp = S.to_device(p, torch.float32)
    ra = S.RaOpts(coarse_stride=p.coarse_stride, coarse_n=p.coarse_n, C=p.ra_C, M=p.ra_M, q=p.ra_q, tol=p.ra_tol)
    theta = torch.as_tensor(p.meta["theta"], dtype=torch.float32, device=DEV).requires_grad_(True)
    mem_t = None if member is None else torch.as_tensor(member, device=DEV)
    opts = S.SolveOpts(tol=0.0, max_sweeps=CAP, local_iters=li)
    V = S.HJBSolve.apply(torch.exp(theta), dp, mem_t, ra, opts, 0.0, li)
    obs_t = torch.as_tensor(obs, device=DEV)
    Vobs_t = torch.as_tensor(Vobs, dtype=torch.float32, device=DEV)
    loss = ((V[obs_t] - Vobs_t) ** 2).sum()
    loss.backward()
    grad = theta.grad.detach().cpu().numpy().astype(np.float64)
    th = p.meta["theta"]
    rng = np.random.Generator(np.random.PCG64(705))
    eps = 1e-6
    for _ in range(4):
        d = rng.normal(size=p.N)
        fd = (loss_o(th + eps * d) - loss_o(th - eps * d)) / (2 * eps)
        an = float(grad @ d)
        say(f"  {mode} {interp} local {li}: fd {fd:.6e} adjoint {an:.6e} "
            f"rel {abs(fd - an) / abs(fd):.2e}")
        assert abs(fd - an) <= 1e-3 * abs(fd)


VARIANTS = {"swirl": dict(swirl=0.5), "axes": dict(axis_speed=True)}


@pytest.mark.parametrize("li", LOCAL)
@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4), (torch.float64, 1e-12)])
@pytest.mark.parametrize("variant", list(VARIANTS))
def test_adjoint_drift_and_axis_speed(variant, dtype, tol, li):
    """Feet shifted by a per-node drift, or stretched by per-axis speed factors:
    the same bars as the plain adjoint."""
    p = W.c5_adjoint(n=129, n_obs=1500, **VARIANTS[variant])
    say("case: adjoint", variant, dtype, "local", li)
    V, pol, _, _ = O.solve(p)
    Vt, _, _, _ = O.solve(p.with_(cost=np.exp(p.meta["theta_true"])))
    obs = p.meta["obs"]
    gV = _obs_grad(p, V, Vt[obs], obs)
    _, dLdl_o, it_o, _ = O.adjoint(p, pol, gV)
    dp = S.to_device(p, dtype)
    dLdl, st = S.adjoint(dp, torch.as_tensor(pol_u8(pol), device=DEV),
                         torch.as_tensor(gV, dtype=dtype, device=DEV),
                         tol=gpu_tol(gV, dtype), local_iters=li)
    err = rel_l2(dLdl.cpu().numpy().astype(np.float64), dLdl_o)
    say("  rel l2", err, "launches", st["sweeps_max"], "oracle iters", it_o)
    assert st["converged"]
    assert err <= tol


def test_adjoint_isa_swirl():
    """Sets of the reconstruction with a drift; per-set adjoints summed."""
    p = W.c5_adjoint(n=129, n_obs=1500, swirl=0.5)
    say("case: isa adjoint with drift")
    Vbar, owner, rec, Vs, _ = I.isa(p)
    _, pols, _ = I.solve_subdomains(p, rec.member, want_policy=True)
    Vt = I.isa(p.with_(cost=np.exp(p.meta["theta_true"])))[0]
    obs = p.meta["obs"]
    gV = _obs_grad(p, Vbar, Vt[obs], obs)
    dLdl_o, _ = I.adjoint_isa(p, rec.member, pols, owner, gV)
    dp = S.to_device(p, torch.float32)
    pol_t = torch.as_tensor(np.concatenate([pol_u8(q) for q in pols]), device=DEV)
    dLdl, st = S.adjoint(dp, pol_t, torch.as_tensor(gV, dtype=torch.float32, device=DEV),
                         member=torch.as_tensor(rec.member, device=DEV),
                         owner=torch.as_tensor(owner, device=DEV), tol=0.0, local_iters=4)
    err = rel_l2(dLdl.cpu().numpy().astype(np.float64), dLdl_o)
    say("  rel l2", err, "launches", st["sweeps_max"])
    assert err <= 1e-4


def test_adjoint_vdp_drift_field():
    """Van der Pol dynamics (drift larger than the control), 257^2, a dense g."""
    p = W.vdp_problem(257, split=1)
    say("case: adjoint vdp 257")
    V, pol, _, _ = O.solve(p)
    gV = np.random.Generator(np.random.PCG64(11)).normal(size=p.N)
    _, dLdl_o, _, _ = O.adjoint(p, pol, gV)
    dp = S.to_device(p, torch.float32)
    for li in LOCAL:
        dLdl, st = S.adjoint(dp, torch.as_tensor(pol_u8(pol), device=DEV),
                             torch.as_tensor(gV, dtype=torch.float32, device=DEV),
                             tol=0.0, local_iters=li)
        err = rel_l2(dLdl.cpu().numpy().astype(np.float64), dLdl_o)
        say("  local", li, "rel l2", err, "launches", st["sweeps_max"])
        assert st["converged"]
        assert err <= 1e-4


def test_autograd_gradient_with_drift_against_fd():
    """theta -> V with a drift (GPU FP32, tiles) -> loss; gradient against central
    differences of the oracle's FP64 loss."""
    p = W.c5_adjoint(n=65, n_obs=300, swirl=0.5)
    obs = p.meta["obs"]
    Vobs = O.solve(p.with_(cost=np.exp(p.meta["theta_true"])))[0][obs]

    def loss_o(theta):
        return float(np.sum((O.solve(p.with_(cost=np.exp(theta)))[0][obs] - Vobs) ** 2))

    dp = S.to_device(p, torch.float32)
    ra = S.RaOpts(coarse_stride=p.coarse_stride, coarse_n=p.coarse_n, C=p.ra_C, M=p.ra_M, q=p.ra_q, tol=p.ra_tol)
    theta = torch.as_tensor(p.meta["theta"], dtype=torch.float32, device=DEV).requires_grad_(True)
    opts = S.SolveOpts(tol=0.0, max_sweeps=CAP, local_iters=4)
    V = S.HJBSolve.apply(torch.exp(theta), dp, None, ra, opts, 0.0, 4)
    loss = ((V[torch.as_tensor(obs, device=DEV)]
             - torch.as_tensor(Vobs, dtype=torch.float32, device=DEV)) ** 2).sum()
    loss.backward()
    grad = theta.grad.detach().cpu().numpy().astype(np.float64)
    th = p.meta["theta"]
    rng = np.random.Generator(np.random.PCG64(706))
    eps = 1e-6
    for _ in range(4):
        d = rng.normal(size=p.N)
        fd = (loss_o(th + eps * d) - loss_o(th - eps * d)) / (2 * eps)
        an = float(grad @ d)
        say(f"  fd {fd:.6e} adjoint {an:.6e} rel {abs(fd - an) / abs(fd):.2e}")
        assert abs(fd - an) <= 1e-3 * abs(fd)


# --------------------------------------------------- gather tiles, determinism
@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4), (torch.float64, 1e-12)])
def test_adjoint_jacobi_mode_is_deterministic(dtype, tol):
    """local_iters = 0 (Jacobi gather over tiles, no atomics): two calls give the
    same bits, global and with sets; both match the oracle's adjoint."""
    p = W.c5_adjoint(n=129, n_obs=1500)
    say("case: deterministic adjoint", dtype)
    Vbar, owner, rec, Vs, _ = I.isa(p)
    _, pols, _ = I.solve_subdomains(p, rec.member, want_policy=True)
    gV = np.random.Generator(np.random.PCG64(17)).normal(size=p.N)
    dLdl_o, _ = I.adjoint_isa(p, rec.member, pols, owner, gV)
    dp = S.to_device(p, dtype)
    pol_t = torch.as_tensor(np.concatenate([pol_u8(q) for q in pols]), device=DEV)
    args = dict(member=torch.as_tensor(rec.member, device=DEV),
                owner=torch.as_tensor(owner, device=DEV), tol=0.0, local_iters=0)
    g_t = torch.as_tensor(gV, dtype=dtype, device=DEV)
    a, st = S.adjoint(dp, pol_t, g_t, **args)
    b, _ = S.adjoint(dp, pol_t, g_t, **args)
    assert st["converged"]
    assert torch.equal(a, b)
    err = rel_l2(a.cpu().numpy().astype(np.float64), dLdl_o)
    say("  rel l2", err, "launches", st["sweeps_max"])
    assert err <= tol


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_adjoint_relative_tolerance(dtype):
    """A negative tol is relative to max |dL/dV|, taken on the device and rounded
    down to a power of two: the same stopping threshold as that absolute tol
    computed on the host, so the Jacobi iterates (deterministic mode) stop at the
    same launch with the same bits."""
    p = W.c5_adjoint(n=65, n_obs=300)
    say("case: relative adjoint tolerance", dtype)
    V, pol = O.solve(p)[:2]
    gV = np.random.Generator(np.random.PCG64(23)).normal(size=p.N)
    dp = S.to_device(p, dtype)
    g_t = torch.as_tensor(gV, dtype=dtype, device=DEV)
    pol_t = torch.as_tensor(pol_u8(pol), device=DEV)
    rtol = 1e-5
    scale = float(np.abs(g_t.cpu().numpy().astype(np.float64)).max())
    m, ex = math.frexp(rtol * scale)
    tol_abs = math.ldexp(0.5, ex)
    assert tol_abs <= rtol * scale < 2 * tol_abs
    a, sa = S.adjoint(dp, pol_t, g_t, tol=-rtol, local_iters=0)
    b, sb = S.adjoint(dp, pol_t, g_t, tol=tol_abs, local_iters=0)
    assert sa["converged"] and sb["converged"]
    assert sa["sweeps_max"] == sb["sweeps_max"]
    assert torch.equal(a, b)


def _adjoint_3d(n=25, seed=3):
    p = W.c3_aniso3d(n=n, m=32, n_balls=3, r=0.15)
    th = np.random.Generator(np.random.PCG64(seed)).normal(0.0, 0.1, p.N)
    return p.with_(cost=W.f32(np.exp(th)), v_ghost=2.0)


@pytest.mark.parametrize("li", LOCAL)
@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4), (torch.float64, 1e-12)])
def test_adjoint_3d_tiles(dtype, tol, li):
    """3D gather tiles (8x8x4 nodes, halo as the feet need), Jacobi and
    block-asynchronous, against the oracle's adjoint; with sets too."""
    p = _adjoint_3d()
    say("case: 3d adjoint tiles", dtype, "local", li)
    V, pol, _, _ = O.solve(p)
    gV = np.random.Generator(np.random.PCG64(19)).normal(size=p.N)
    _, dLdl_o, _, _ = O.adjoint(p, pol, gV)
    dp = S.to_device(p, dtype)
    dLdl, st = S.adjoint(dp, torch.as_tensor(pol_u8(pol), device=DEV),
                         torch.as_tensor(gV, dtype=dtype, device=DEV), tol=0.0, local_iters=li)
    err = rel_l2(dLdl.cpu().numpy().astype(np.float64), dLdl_o)
    say("  global rel l2", err, "launches", st["sweeps_max"])
    assert st["converged"] and err <= tol
    Vbar, owner, rec, Vs, _ = I.isa(p)
    _, pols, _ = I.solve_subdomains(p, rec.member, want_policy=True)
    dLdl_o, _ = I.adjoint_isa(p, rec.member, pols, owner, gV)
    dLdl, st = S.adjoint(dp, torch.as_tensor(np.concatenate([pol_u8(q) for q in pols]), device=DEV),
                         torch.as_tensor(gV, dtype=dtype, device=DEV),
                         member=torch.as_tensor(rec.member, device=DEV),
                         owner=torch.as_tensor(owner, device=DEV), tol=0.0, local_iters=li)
    err = rel_l2(dLdl.cpu().numpy().astype(np.float64), dLdl_o)
    say("  sets rel l2", err, "launches", st["sweeps_max"])
    assert st["converged"] and err <= tol


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-4), (torch.float64, 1e-12)])
def test_adjoint_long_feet_scatter_path(dtype, tol):
    """Feet longer than the tiles' halo (speed 8.5, so 9 cells in 2D) take the
    whole-grid Jacobi scatter: same bars."""
    p = W.c5_adjoint(n=97, n_obs=500)
    p = p.with_(speed=W.f32(np.full(p.N, 8.5)))
    say("case: adjoint scatter path", dtype)
    V, pol, _, _ = O.solve(p)
    gV = np.random.Generator(np.random.PCG64(23)).normal(size=p.N)
    _, dLdl_o, _, _ = O.adjoint(p, pol, gV)
    dp = S.to_device(p, dtype)
    for li in LOCAL:
        dLdl, st = S.adjoint(dp, torch.as_tensor(pol_u8(pol), device=DEV),
                             torch.as_tensor(gV, dtype=dtype, device=DEV), tol=0.0,
                             local_iters=li)
        err = rel_l2(dLdl.cpu().numpy().astype(np.float64), dLdl_o)
        say("  local", li, "rel l2", err, "launches", st["sweeps_max"])
        assert st["converged"] and err <= tol
