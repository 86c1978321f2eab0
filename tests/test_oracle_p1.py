"""Pins of the oracle's P1 (Kuhn simplex) interpolation (no GPU).

The scheme of Sec. 3 interpolates piecewise linearly on a simplicial grid.  Here
every grid cell is split into its Kuhn simplices, the simplex of a point fixed by
the order of its fractional coordinates; the oracle evaluates the interpolant as
nested one-dimensional interpolations.  The pins below come from outside that
code: a closed form of P1 applied to x*y, exact rational policy iteration with
the barycentric weights (2D and 3D), the strip example's closed form (a field
that depends on x1 alone interpolates the same way on every simplex), monotonicity
and exact reproduction of a power-of-two constant."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import tiny


def _one_control(n, a, seed):
    """n x n grid on [0, n-1]^2 (index units = coordinates, h = dx = 1), one control
    a, random per-node speed so the feet land at assorted fractions, l = 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tid = np.full(n * n, -1, dtype=np.int8)
    tid[0] = 0
    speed = W.f32(rng.uniform(0.05, 1.9, n * n))
    return W.Problem(name="p1_probe", dim=2, n=(n, n), lo=(0.0, 0.0),
                     hi=(float(n - 1), float(n - 1)), velocity=np.array([a]), target=tid,
                     n_comp=1, speed=speed, v_ghost=1.0, interp="p1")


def _interp_values(p, V):
    """I[V] at each node's foot, read back from one application of T with a single
    control and l = 1: T(V)_j = beta I[V](foot_j) + w."""
    TV, _ = O.apply_T(p, V, fixed=np.zeros(p.N, dtype=np.uint8))
    beta, w = O.scheme_constants(p.lam, p.step, p.disc)
    return (TV - w) / beta


@pytest.mark.parametrize("a,seed", [((0.6, 0.35), 1), ((-0.45, 0.8), 2), ((0.3, -0.9), 3)])
def test_p1_of_xy_closed_form(a, seed):
    """P1 of x*y on the Kuhn simplices: with the foot u = p + (fx, fy) in a cell,
    the interpolant is u0 u1 + min(fx, fy) (1 - max(fx, fy)).  Q1 would give
    u0 u1 exactly and the other diagonal a different correction, so a wrong
    simplex, vertex or weight fails here."""
    n = 12
    p = _one_control(n, a, seed)
    X = W.node_coords(p.n, p.lo, p.hi)
    V = X[:, 0] * X[:, 1]
    got = _interp_values(p, V)
    c = p.speed.astype(np.float64)
    u = X + np.outer(c, np.asarray(a, dtype=np.float64))
    inside = ((u >= 0) & (u <= n - 1)).all(axis=1)
    fl = np.floor(u)
    f = u - fl
    exact = u[:, 0] * u[:, 1] + np.minimum(f[:, 0], f[:, 1]) * (1 - np.maximum(f[:, 0], f[:, 1]))
    assert inside.sum() > 0.5 * p.N
    assert np.abs(got[inside] - exact[inside]).max() <= 1e-12 * (n * n)
    # and Q1 on the same feet reproduces x*y itself
    q1 = _interp_values(p.with_(interp="q1"), V)
    assert np.abs(q1[inside] - (u[inside, 0] * u[inside, 1])).max() <= 1e-12 * (n * n)


def test_p1_affine_fields_reproduced():
    """Both interpolants are exact on affine fields."""
    n = 10
    p = _one_control(n, (0.55, -0.7), 5)
    X = W.node_coords(p.n, p.lo, p.hi)
    V = 3.0 - 0.25 * X[:, 0] + 0.5 * X[:, 1]
    u = X + np.outer(p.speed.astype(np.float64), [0.55, -0.7])
    inside = ((u >= 0) & (u <= n - 1)).all(axis=1)
    got = _interp_values(p, V)
    assert np.abs(got[inside] - (3.0 - 0.25 * u[inside, 0] + 0.5 * u[inside, 1])).max() <= 1e-12


def test_p1_power_of_two_constant_exact_and_monotone():
    """A constant field of 2 (the ghost value) is reproduced bit for bit, and T is
    monotone: V <= V' node by node gives T(V) <= T(V')."""
    p = W.c2_multitarget(n=33, m=16, n_disks=2, r=0.1, seed_field=7, seed_disks=8)
    p = p.with_(interp="p1", v_ghost=2.0)
    beta, w = O.scheme_constants(p.lam, p.step, p.disc)
    TV, _ = O.apply_T(p, np.full(p.N, 2.0), fixed=np.zeros(p.N, dtype=np.uint8))
    assert (TV == 2.0 * beta + w).all()
    rng = np.random.Generator(np.random.PCG64(9))
    V = rng.uniform(0.0, 2.0, p.N)
    Vp = V + rng.uniform(0.0, 1e-3, p.N) * (rng.random(p.N) < 0.5)
    T1, _ = O.apply_T(p, V)
    T2, _ = O.apply_T(p, Vp)
    assert (T2 >= T1).all()


def _tiny_2d(n, m, seed, **kw):
    p = W.c2_multitarget(n=n, m=m, n_disks=2, r=0.05, seed_field=seed, seed_disks=seed + 1)
    return p.with_(interp="p1", **kw)


CASES = [
    ("2d_n7_m8", lambda: _tiny_2d(7, 8, 11)),
    ("2d_n9_m16", lambda: _tiny_2d(9, 16, 21)),
    ("2d_m7_ghost2", lambda: _tiny_2d(9, 7, 31, v_ghost=2.0)),
    ("3d_n4_m10", lambda: W.c3_aniso3d(n=4, m=10, n_balls=1, r=0.5).with_(interp="p1")),
    ("2d_vdp_drift_n9", lambda: W.vdp_problem(9, split=1, n_a=5).with_(interp="p1")),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_p1_jacobi_matches_exact_policy_iteration(name, mk):
    """The oracle's Jacobi fixed point with P1 equals the exact fixed point found by
    policy iteration with rational barycentric weights on the Kuhn simplices."""
    p = mk()
    Vx, pol_x, _ = tiny.policy_iteration(p)
    V, pol, _, res = O.solve(p)
    assert res == 0.0
    Vf = np.array([float(v) for v in Vx])
    assert np.abs(Vf - V).max() <= 1e-13
    gaps = tiny.candidate_gaps(p, Vx)
    clear = (pol_x >= 0) & (gaps > 1e-12)
    assert (pol[clear] == pol_x[clear]).all()
    # and the P1 solution differs from the Q1 one (the pin is not vacuous)
    assert np.abs(O.solve(p.with_(interp="q1"))[0] - V).max() > 1e-6


@pytest.mark.parametrize("delta", [1.0, 0.1])
def test_p1_strip_closed_form(delta):
    """Strip example (Sec. 3, Example 3.1): V depends on x1 only, and such a field
    interpolates the same on every Kuhn simplex as under Q1, so the P1 solution
    equals the closed form (1 - exp(-delta (1 - |x1|)))/delta at the nodes."""
    n = 21
    p = W.strip_problem(n, delta).with_(interp="p1")
    V, _, _, res = O.solve(p)
    assert res == 0.0
    X = W.grid_axes(p.n, p.lo, p.hi)[0]
    exact = (1.0 - np.exp(-delta * (1.0 - np.abs(X)))) / delta
    assert np.abs(V.reshape(n, n) - exact[None, :]).max() <= 1e-13


def test_p1_adjoint_matches_linear_solve():
    """The policy stencil with P1 (vertices and barycentric weights) reproduces the
    P1 fixed point, and the adjoint's dot product with the tangent holds."""
    p = W.c5_adjoint(n=33, n_obs=100).with_(interp="p1")
    V, pol, _, _ = O.solve(p)
    cidx, wts = O.policy_stencil(p, pol)
    assert np.allclose(wts.sum(axis=1)[pol >= 0], 1.0, atol=1e-15, rtol=0)
    assert (wts >= 0).all()
    rng = np.random.Generator(np.random.PCG64(4))
    gV = rng.normal(size=p.N)
    dl = rng.normal(size=p.N)
    _, dLdl, _, _ = O.adjoint(p, pol, gV)
    Vdot, _ = O.tangent(p, pol, dl)
    lhs, rhs = float(np.dot(dLdl, dl)), float(np.dot(gV, Vdot))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
    # fixed point through the stencil: V_j = beta sum w V(corner) + w l_j
    beta, w = O.scheme_constants(p.lam, p.step, p.disc)
    free = np.flatnonzero(pol >= 0)
    vals = np.where(cidx[free] >= 0, V[np.maximum(cidx[free], 0)], p.v_ghost)
    rec = beta * (wts[free] * vals).sum(axis=1) + w * p.cost[free]
    assert np.abs(rec - V[free]).max() <= 1e-12
