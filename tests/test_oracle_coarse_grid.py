"""Pins of the oracle's coarse grid K (RA, Sec. 3-4) when K is any uniform grid on
the box, nested in the fine grid or not (Sec. 4 only asks that both cover the
domain).  No GPU."""
from fractions import Fraction
import itertools

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import isa as I


def _multilinear(X):
    """A function in the Q1 space with distinct coefficients on every monomial, so
    a swapped axis, a wrong fraction or a wrong corner changes the result."""
    x = X[:, 0]
    y = X[:, 1]
    f = 0.3 + 1.7 * x - 0.9 * y + 0.4 * x * y
    if X.shape[1] == 3:
        z = X[:, 2]
        f = f + 0.8 * z - 0.5 * x * z + 0.25 * y * z + 0.6 * x * y * z
    return f


@pytest.mark.parametrize("n,nK", [((13, 10), (5, 7)), ((41, 41), (15, 15)), ((9, 9), (5, 5)),
                                  ((7, 9, 6), (4, 5, 3)), ((12, 11), (12, 11))])
def test_q1_sampling_is_exact_on_multilinear_fields(n, nK):
    """Q1 interpolation reproduces a multilinear function exactly (up to rounding),
    so the sampled coarse field equals the function at the coarse nodes."""
    lo = tuple(-1.0 for _ in n)
    hi = tuple(1.0 for _ in n)
    fine = _multilinear(W.node_coords(n, lo, hi))
    got = I.sample_q1(fine, n, nK)
    want = _multilinear(W.node_coords(nK, lo, hi))
    assert np.abs(got - want).max() <= 1e-13


def test_nested_coarse_counts_equal_the_stride_grid():
    """Given as node counts, a nested coarse grid yields exactly (bit for bit) the
    coarse problem of the stride: coincident nodes copy the fine data."""
    base = W.c2_multitarget(n=97, m=16)
    rng = np.random.Generator(np.random.PCG64(9))
    p = base.with_(cost=W.f32(np.exp(rng.normal(0, 0.3, base.N))),
                   g=W.f32(rng.uniform(0, 0.1, base.N)),
                   drift=W.f32(rng.normal(0, 0.2, (base.N, 2))))
    a = I.coarse_problem(p.with_(coarse_stride=4))
    b = I.coarse_problem(p.with_(coarse_n=(25, 25)))
    assert a.n == b.n == (25, 25) and a.h == b.h
    for f in ("speed", "cost", "g", "target", "drift"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    sl = np.asarray(p.speed).reshape(97, 97)[::4, ::4].reshape(-1)
    assert np.array_equal(a.speed, sl)


def _nearest_fine(k, n, nK):
    """Nearest fine index to coarse index k by exact rational rounding (ties up)."""
    return int(Fraction(k * (n - 1), nK - 1) + Fraction(1, 2))


@pytest.mark.parametrize("n,nK,seed", [((12, 11), (5, 4), 1), ((30, 17), (9, 8), 2),
                                       ((7, 6, 9), (4, 4, 5), 3)])
def test_coarse_targets_and_exit_costs_from_the_nearest_fine_node(n, nK, seed):
    dim = len(n)
    N = int(np.prod(n))
    rng = np.random.Generator(np.random.PCG64(seed))
    tid = rng.integers(-1, 3, N).astype(np.int8)
    g = W.f32(rng.uniform(0, 1, N))
    base = W.c1_eikonal(5) if dim == 2 else W.c3_aniso3d(n=4, m=10, n_balls=1, r=0.5)
    p = base.with_(n=n, lo=(-1.0,) * dim, hi=(1.0,) * dim, target=tid, n_comp=3, g=g,
                   speed=None, cost=None, drift=None, coarse_n=nK)
    pk = I.coarse_problem(p)
    T = tid.reshape(tuple(reversed(n)))
    G = g.reshape(tuple(reversed(n)))
    for ck in itertools.product(*[range(nK[d]) for d in range(dim)]):
        jk = 0
        stride = 1
        for d in range(dim):
            jk += ck[d] * stride
            stride *= nK[d]
        near = tuple(_nearest_fine(ck[d], n[d], nK[d]) for d in range(dim))
        assert pk.target[jk] == T[tuple(reversed(near))]
        assert pk.g[jk] == G[tuple(reversed(near))]


def test_component_without_coarse_node_goes_to_the_nearest_one():
    """A one-node target between coarse nodes is placed at the coarse node nearest
    to it; an occupied coarse node is not taken over."""
    n, nK = (12, 11), (5, 4)
    N = n[0] * n[1]
    tid = np.full(N, -1, dtype=np.int8)
    tid[5 + 12 * 3] = 0          # fine (5, 3): coarse coordinates (20/11, 9/10) -> (2, 1)
    tid[10 + 12 * 8] = 1         # fine (10, 8): (40/11, 24/10) -> (4, 2)
    p = W.c1_eikonal(5).with_(n=n, target=tid, n_comp=2, coarse_n=nK)
    pk = I.coarse_problem(p)
    want = np.full(nK[0] * nK[1], -1, dtype=np.int8)
    want[2 + 5 * 1] = 0
    want[4 + 5 * 2] = 1
    assert np.array_equal(pk.target, want)


def test_coarse_step_scales_with_the_largest_spacing_ratio():
    p = W.c2_multitarget(n=97, m=16).with_(coarse_n=(35, 35))
    pk = I.coarse_problem(p)
    assert pk.h == p.step * (96 / 34)
    assert pk.n == (35, 35) and pk.N == 35 * 35


def test_box_distance_isa_with_the_papers_15_point_coarse_grid():
    """Sec. 4.1, distance function with the 4-way split and a coarse grid of 15^2
    points (not nested in 101^2): the projected sets contain the four exact
    triangles and the ISA reproduces the global solution."""
    n = 101
    p = W.box_distance_problem(n, split=4).with_(coarse_n=(15, 15), ra_C=0.25, ra_M=0.25)
    Vg, _, _, _ = O.solve(p)
    Vbar, owner, rec, Vs, _ = I.isa(p)
    assert np.abs(Vbar - Vg).max() <= 1e-14
    X = W.node_coords(p.n, p.lo, p.hi)
    x1, x2 = X[:, 0], X[:, 1]
    dist = np.stack([1 + x2, 1 - x1, 1 - x2, 1 + x1], axis=1)
    dmin = dist.min(axis=1)
    for i in range(4):
        true_set = dist[:, i] <= dmin + 1e-12
        bit = ((rec.member >> i) & 1).astype(bool)
        assert bit[true_set].all(), f"true sub-domain {i} not contained"


def test_multitarget_isa_with_a_non_nested_coarse_grid():
    """Variable speed, 4 disks, 97^2 fine and 35^2 coarse: the ISA is never below
    the global solution and equals it wherever the global optimal dependencies
    stay in the set (the discrete Proposition 2.1)."""
    p = W.c2_multitarget(n=97, m=32).with_(coarse_n=(35, 35))
    Vg, pol, _, _ = O.solve(p)
    Vbar, owner, rec, Vs, _ = I.isa(p)
    assert (Vbar >= Vg - 1e-15).all()
    from tests.test_oracle_invariants import _escape_sets
    esc = _escape_sets(p, pol, rec.member)
    closed_any = np.zeros(p.N, dtype=bool)
    for i in range(p.n_comp):
        ok = (~esc[i]) & (((rec.member >> i) & 1).astype(bool))
        assert np.abs(Vs[i][ok] - Vg[ok]).max(initial=0.0) <= 1e-12
        closed_any |= ok
    assert closed_any.mean() > 0.9
