"""Invariant pins of the FP64 oracle: properties the paper's theorems and the
scheme's structure fix at any size (no GPU)."""
import numpy as np
import pytest
from scipy import ndimage

import oracle as O
import workloads as W
from oracle import isa as I


@pytest.fixture(scope="module")
def c2_small():
    return W.c2_multitarget(n=97, m=32)


@pytest.fixture(scope="module")
def c3_small():
    return W.c3_aniso3d(n=17, m=32, n_balls=3, r=0.15)


@pytest.fixture(scope="module")
def c3_unit():
    return W.c3_aniso3d(n=17, m=32, n_balls=3, r=0.15).with_(speed=None)


def _rand_values(p, seed, lo=0.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    V = rng.uniform(lo, p.v_ghost, p.N)
    V0 = O.initial_values(p)
    fx = O.fixed_mask(p).astype(bool)
    V[fx] = V0[fx]
    return V


@pytest.mark.parametrize("which", ["c2_small", "c3_small"])
def test_contraction_and_monotonicity(which, request):
    """T is a beta-contraction in the sup norm and monotone (Sec. 3: the map
    V -> T(V) 'is shown to be a contraction')."""
    p = request.getfixturevalue(which)
    beta, _ = O.scheme_constants(p.lam, p.step)
    V = _rand_values(p, 1)
    Wv = _rand_values(p, 2)
    TV, _ = O.apply_T(p, V)
    TW, _ = O.apply_T(p, Wv)
    assert np.abs(TV - TW).max() <= beta * np.abs(V - Wv).max() * (1 + 1e-12)
    # monotone: V <= W  =>  T V <= T W
    lo = np.minimum(V, Wv)
    Tlo, _ = O.apply_T(p, lo)
    assert (Tlo <= TV + 1e-15).all() and (Tlo <= TW + 1e-15).all()


def test_iterates_monotone_from_ghost(c2_small):
    """From V^0 = ghost value (a supersolution) the Jacobi iterates decrease
    monotonically, also in floating point, and stay in [0, V_ghost]."""
    p = c2_small
    V = O.initial_values(p)
    prev = V.copy()
    for _ in range(40):
        V, _, _, _ = O.solve(p, V0=prev, max_sweeps=1)
        assert (V <= prev).all()
        prev = V
    Vf, _, _, res = O.solve(p)
    assert res == 0.0
    assert (Vf <= V).all()
    assert Vf.min() >= 0.0 and Vf.max() <= p.v_ghost


def test_fixed_point_residual_is_zero(c2_small):
    """At stagnation V = T(V) exactly."""
    Vf, _, _, _ = O.solve(c2_small)
    TV, _ = O.apply_T(c2_small, Vf)
    assert np.array_equal(TV, Vf)


def test_d4_symmetry_point_target():
    """Point target at the centre with an exactly D4-symmetric control set: V is
    symmetric under the square's symmetries (up to FP accumulation order)."""
    n = 61
    p = W.c1_eikonal(n)
    V, _, _, _ = O.solve(p)
    Vg = V.reshape(n, n)
    for img in (Vg[::-1, :], Vg[:, ::-1], Vg.T, Vg[::-1, ::-1].T):
        assert np.abs(Vg - img).max() <= 1e-14


def test_global_below_auxiliary_min(c2_small):
    """Theorem 2.1, discrete side: every auxiliary value V_i is >= the global
    discrete value, and min_i V_i is >= it too."""
    p = c2_small.with_(coarse_stride=1)
    Vg, _, _, _ = O.solve(p)
    _, _, V_aux, Vmin, _, _ = I.reconstruct_on(p)
    for Vi in V_aux:
        assert (Vi >= Vg - 1e-15).all()
    assert (Vmin >= Vg - 1e-15).all()


def test_reconstruction_covers_and_is_connected(c2_small):
    """I7: every fine node is in some set and Gamma_i is inside set i.  The exact
    discrete sub-domains {V_i = min_k V_k} (fine-grid auxiliary solves) are
    connected (Corollary 2.1: Gamma_i connected => Sigma_i connected) and lie
    inside the reconstructed sets (Sigma_i included in the approximation, Sec. 3).
    The approximations themselves need not be connected: the threshold band may
    also catch a detached near-tie patch."""
    p = c2_small
    rec = I.reconstruct(p)
    assert (rec.member > 0).all()
    tid = np.asarray(p.target)
    _, _, V_aux, V_min, _, _ = I.reconstruct_on(p.with_(coarse_stride=1))
    for i in range(p.n_comp):
        bit = ((rec.member >> i) & 1).astype(bool)
        assert bit[tid == i].all()
        exact = V_aux[i] == V_min
        _, nlab = ndimage.label(exact.reshape(p.shape()))
        assert nlab == 1, f"exact set {i} has {nlab} components"
        assert bit[exact].all()
        lab, _ = ndimage.label(bit.reshape(p.shape()))
        main = lab.reshape(-1)[np.flatnonzero(tid == i)[0]]
        assert (lab.reshape(-1)[exact] == main).all()


def _escape_sets(p, pol, member):
    """Nodes whose global-policy dependency closure leaves set i (per i)."""
    cidx, wts = O.policy_stencil(p, pol)
    out = []
    for i in range(p.n_comp):
        inside = ((member >> i) & 1).astype(bool)
        esc = ~inside
        while True:
            bad = esc[np.where(cidx >= 0, cidx, 0)] & (wts > 0) & (cidx >= 0)
            new = esc | (bad.any(axis=1) & (pol >= 0))
            if np.array_equal(new, esc):
                break
            esc = new
        out.append(esc)
    return out


@pytest.mark.parametrize("which,min_closed", [("c2_small", 0.9), ("c3_unit", 0.1)])
def test_subdomain_exactness(which, min_closed, request):
    """I8, the discrete content of Proposition 2.1 / 4.1: wherever the global
    solution's dependency closure (under its optimal policy) stays inside a set
    containing the node, solving that set alone reproduces the global value; and
    the assembled value is never below the global one.  (In 3D, Q1 interpolation
    spreads dependency closures widely, so fewer nodes are closed.)"""
    p = request.getfixturevalue(which)
    Vg, pol, _, _ = O.solve(p)
    Vbar, owner, rec, Vs, _ = I.isa(p)
    assert (Vbar >= Vg - 1e-15).all()
    esc = _escape_sets(p, pol, rec.member)
    closed_any = np.zeros(p.N, dtype=bool)
    for i in range(p.n_comp):
        ok = (~esc[i]) & (((rec.member >> i) & 1).astype(bool))
        assert np.abs(Vs[i][ok] - Vg[ok]).max(initial=0.0) <= 1e-12
        closed_any |= ok
    assert np.abs(Vbar[closed_any] - Vg[closed_any]).max() <= 1e-12
    assert closed_any.mean() > min_closed


def test_voronoi_partition_equal_disks():
    """Equal point-like targets with unit speed: the owner of a node (argmin of the
    sub-domain values) is its nearest target (Voronoi cell), away from bisectors."""
    n = 81
    p = W.c2_multitarget(n=n, m=32, n_disks=3, r=0.02, seed_disks=77).with_(speed=None)
    Vbar, owner, rec, Vs, _ = I.isa(p)
    X = W.node_coords(p.n, p.lo, p.hi)
    cen = p.meta["centres"]
    d = np.sqrt(((X[:, None, :] - cen[None, :, :]) ** 2).sum(-1))
    ds = np.sort(d, axis=1)
    far = (ds[:, 1] - ds[:, 0]) > 2 * 2.0 * p.dx[0]
    assert (owner[far] == np.argmin(d, axis=1)[far]).all()


def test_isa_error_matches_global_error():
    """Proposition 4.1 / Table 3: the ISA solution's error against the closed form
    is of the same order as the global solve's.  Targets sit on coarse nodes, so
    the coarse auxiliary problems see the same targets as the fine ones."""
    n = 101
    base = W.c1_eikonal(n)
    # three point targets with unit speed: v = 1 - exp(-min_i |x - p_i|)
    tid = np.full(base.N, -1, dtype=np.int8)
    pts = [(24, 32), (76, 52), (40, 80)]
    for i, (a, b) in enumerate(pts):
        tid[a + n * b] = i
    p = base.with_(target=tid, n_comp=3, coarse_stride=4)
    X = W.node_coords(p.n, p.lo, p.hi)
    P = np.array([X[a + n * b] for a, b in pts])
    ex = 1.0 - np.exp(-np.sqrt(((X[:, None, :] - P[None]) ** 2).sum(-1)).min(axis=1))
    Vg, _, _, _ = O.solve(p)
    Vbar, _, _, _, _ = I.isa(p)
    eg, ei = np.abs(Vg - ex).max(), np.abs(Vbar - ex).max()
    assert ei <= eg * 1.05 + 1e-12
    assert ei < 2e-2


def test_inclusion_across_nested_coarse_grids(c2_small):
    """(incap): a coarser grid's reconstructed set contains a finer one's (soft:
    the property is asymptotic; we require it on >= 99% of nodes, with
    delta = 2 dx_K on grids of 13^2 and 25^2 nodes)."""
    p = c2_small.with_(ra_C=0.5, ra_M=0.5)         # n = 97
    sets = []
    for s in (8, 4):
        rec = I.reconstruct(p.with_(coarse_stride=s))
        sets.append(rec.member)
    coarse, fine = sets
    for i in range(p.n_comp):
        c = ((coarse >> i) & 1).astype(bool)
        f = ((fine >> i) & 1).astype(bool)
        assert (c | ~f).mean() >= 0.99


@pytest.mark.parametrize("which", ["c2_gs", "c3_gs"])
def test_any_update_order_reaches_the_jacobi_fixed_point(which):
    """The FP64 evaluation of T is monotone in every node value and maps the
    initial values (ghost value 1, a power of two) to values no larger, exactly.
    From that supersolution every order of updates decreases to the greatest
    floating-point fixed point below it: a block Gauss-Seidel order (three
    interleaved families of 8^d blocks, updated in turn with the others held)
    ends on Jacobi's fixed point bit for bit."""
    p = (W.c2_multitarget(n=65, m=16) if which == "c2_gs"
         else W.c3_aniso3d(n=13, m=16, n_balls=2, r=0.2))
    Vj, _, _, _ = O.solve(p)
    V = O.initial_values(p)
    TV0, _ = O.apply_T(p, V)
    assert (TV0 <= V).all()
    fx = O.fixed_mask(p).astype(bool)
    X = np.stack(np.unravel_index(np.arange(p.N), tuple(reversed(p.n))), axis=1)
    family = (X // 8).sum(axis=1) % 3
    for _ in range(100000):
        changed = False
        for b in range(3):
            hold = (fx | (family != b)).astype(np.uint8)
            Vn, _ = O.apply_T(p, V, fixed=hold)
            changed |= not np.array_equal(Vn, V)
            assert (Vn <= V).all()
            V = Vn
        if not changed:
            break
    assert np.array_equal(V, Vj)
