"""Pins of the oracle's differential-game operator (paper Sec. 2-3: the maximum
over the evader's choices b_l of the minimum over the pursuer's controls a_k, with
dynamics drift(x) + S(x)(a_k - b_l)) and of per-axis speed factors S(x) =
diag(c_1(x), .., c_d(x)).  No GPU.

* closed forms where every foot lands on a node (a game along one axis), one with a
  symmetric evader set (fixes max against min) and one with a one-sided evader
  (fixes the sign of b);
* exact brute force on tiny grids: the game value is the pointwise maximum over the
  evader's stationary strategies of the exact control-problem values they leave;
* reductions: an evader whose only choice is 0 is the control problem, bit for bit;
  equal per-axis factors are the scalar speed, bit for bit;
* monotonicity in the control sets; the sub-domain property of the ISA for games.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import isa as I
from oracle import tiny


def _strip_closed_form(p, cells_per_step):
    beta, w = O.scheme_constants(p.lam, p.step)
    i = np.arange(p.N) % p.n[0]
    k = np.ceil((i - 3) / cells_per_step)
    return np.where(i < 4, 0.0, w * (1.0 - beta ** k) / (1.0 - beta))


def test_symmetric_evader_slows_the_pursuer():
    """a in {-e1, +e1}, b in {-e1/2, +e1/2}, h = 2 dx: the evader's best choice
    pushes away from the target, so each step gains (1 - 1/2) h = one cell:
    V_i = w (1 - beta^(i-3))/(1 - beta).  With min in place of max the pursuer would
    gain three cells a step."""
    p = W.strip_game_problem(41)
    V, _, _, _ = O.solve(p)
    assert np.abs(V - _strip_closed_form(p, 1)).max() <= 1e-15
    assert np.abs(V - _strip_closed_form(p, 3)).max() > 0.1


def test_one_sided_evader_fixes_the_sign_of_b():
    """b = +e1/2 only: f = a - b moves the pursuer by (-1 - 1/2) h = three cells a
    step toward the target (with a + b it would be one cell)."""
    p = W.strip_game_problem(41, evader=(0.5,))
    V, _, _, _ = O.solve(p)
    assert np.abs(V - _strip_closed_form(p, 3)).max() <= 1e-15
    assert np.abs(V - _strip_closed_form(p, 1)).max() > 0.1


def _tiny_game_2d():
    X = W.node_coords((4, 3), (-1.0, -1.0), (1.0, 1.0))
    tid = np.full(12, -1, np.int8)
    tid[[0, 7]] = 0
    return W.Problem(name="tiny_game_2d", dim=2, n=(4, 3), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                     velocity=W.circle_controls(3, 1.0),
                     velocity_b=np.array([[0.4, 0.1], [-0.2, 0.35]]), target=tid, n_comp=1,
                     speed=W.f32(np.stack([1 + 0.3 * X[:, 1], 1 - 0.2 * X[:, 0]], 1)),
                     cost=W.f32(1 + 0.5 * X[:, 0] ** 2), h=0.55, v_ghost=2.0)


def _tiny_game_3d():
    n = (3, 3, 2)
    X = W.node_coords(n, (-1.0,) * 3, (1.0,) * 3)
    N = 18
    tid = np.full(N, -1, np.int8)
    tid[[4, 9, 11, 13, 15, 16, 17]] = 0         # 11 free nodes would be 2048 strategies
    tid[[0, 2]] = 0
    vel = np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.2], [-0.6, 0.3, -0.7]])
    return W.Problem(name="tiny_game_3d", dim=3, n=n, lo=(-1.0,) * 3, hi=(1.0,) * 3,
                     velocity=vel, velocity_b=np.array([[0.3, 0.2, -0.1], [-0.25, 0.0, 0.3]]),
                     target=tid, n_comp=1,
                     speed=W.f32(np.stack([1 + 0.2 * X[:, 2], 0.9 + 0.1 * X[:, 0],
                                           1.1 - 0.2 * X[:, 1]], 1)),
                     h=0.6, v_ghost=2.0)


@pytest.mark.parametrize("make", [_tiny_game_2d, _tiny_game_3d])
def test_game_value_by_brute_force(make):
    p = make()
    Vx, n_strat, attained = tiny.game_value(p)
    Vx = np.array([float(x) for x in Vx])
    V, _, _, _ = O.solve(p)
    assert n_strat >= 64
    assert attained                 # one stationary evader strategy is optimal everywhere
    assert np.abs(V - Vx).max() <= 1e-13
    # the pin sees the evader and the per-axis factors: without either, values move
    ctrl = O.solve(p.with_(velocity_b=None))[0]
    swapped = O.solve(p.with_(speed=np.ascontiguousarray(np.asarray(p.speed)[:, ::-1])))[0]
    assert np.abs(ctrl - Vx).max() > 1e-3
    assert np.abs(swapped - Vx).max() > 1e-3


def test_zero_evader_is_the_control_problem():
    p = W.c2_multitarget(n=65, m=16)
    V0, pol0, s0, _ = O.solve(p)
    V1, pol1, s1, _ = O.solve(p.with_(velocity_b=np.zeros((1, 2))))
    assert np.array_equal(V0, V1) and np.array_equal(pol0, pol1) and s0 == s1


def test_equal_axis_factors_are_the_scalar_speed():
    p = W.c2_multitarget(n=65, m=16)
    c = np.asarray(p.speed)
    V0, pol0, _, _ = O.solve(p)
    V1, pol1, _, _ = O.solve(p.with_(speed=np.stack([c, c], axis=1)))
    assert np.array_equal(V0, V1) and np.array_equal(pol0, pol1)


def test_per_axis_speed_closed_form():
    """Control problem, a in {+-e1, +-e2}, speed factors (2, 1), h = dx, target the
    four leftmost columns: two cells a step, V_i = w (1 - beta^ceil((i-3)/2))/(1-beta).
    The factors swapped would give one cell a step."""
    n = 33
    X = W.node_coords((n, 5), (-1.0, -1.0), (1.0, 1.0))
    i0 = np.arange(X.shape[0]) % n
    base = W.Problem(name="axes", dim=2, n=(n, 5), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                     velocity=np.array([[-1.0, 0.0], [1.0, 0.0], [0.0, 1.0], [0.0, -1.0]]),
                     target=np.where(i0 < 4, 0, -1).astype(np.int8), n_comp=1, v_ghost=4.0)
    fac = np.tile([2.0, 1.0], (base.N, 1))
    V = O.solve(base.with_(speed=fac))[0]
    assert np.abs(V - _strip_closed_form(base, 2)).max() <= 1e-15
    Vs = O.solve(base.with_(speed=np.ascontiguousarray(fac[:, ::-1])))[0]
    assert np.abs(Vs - _strip_closed_form(base, 1)).max() <= 1e-15


def test_values_are_monotone_in_the_control_sets():
    """More evader choices never lower the value; more pursuer controls never raise it."""
    p = W.pursuit_evasion_problem(33, split=1, m_a=12, m_b=4)
    V, _, _, _ = O.solve(p)
    Vb = O.solve(p.with_(velocity_b=W.circle_controls(8, 0.5, centre=True)))[0]
    Va = O.solve(p.with_(velocity=W.circle_controls(24, 1.0)))[0]
    assert (Vb >= V).all() and (Vb > V).any()
    assert (Va <= V).all() and (Va < V).any()


def _best_responses(p, V):
    """Per free node and evader choice l, the table row l m + k of the pursuer's
    first best answer at V."""
    vb = np.asarray(p.velocity_b)
    rows = []
    for l in range(vb.shape[0]):
        _, pol = O.apply_T(p.with_(velocity_b=vb[l:l + 1]), V)
        rows.append(np.where(pol >= 0, l * p.m + pol, -1))
    return np.stack(rows, axis=1)


def test_isa_sub_domain_property_for_a_game():
    """Pursuit-evasion, 4 capture arcs: the assembled value is never below the
    global one, and a set reproduces the global value wherever the dependency
    closure under every evader choice and the pursuer's best answer to it stays in
    the set (for such nodes the set's value is bounded by a contraction of itself).
    Closures that follow every evader choice are wide, so few nodes qualify; off
    them the discrete max-min does not commute with the minimum over the targets,
    and the assembled value sits above the global one by a discretisation-size
    amount."""
    p = W.pursuit_evasion_problem(41, split=4, m_a=16, m_b=4).with_(coarse_n=(21, 21))
    Vg, _, _, _ = O.solve(p)
    Vbar, owner, rec, Vs, _ = I.isa(p)
    assert (Vbar >= Vg - 1e-15).all()
    resp = _best_responses(p, Vg)
    deps = []
    for l in range(resp.shape[1]):
        cidx, wts = O.policy_stencil(p, resp[:, l])
        deps.append(np.where(wts > 0, cidx, -1))
    deps = np.concatenate(deps, axis=1)
    free = resp[:, 0] >= 0
    closed_any = np.zeros(p.N, dtype=bool)
    for i in range(p.n_comp):
        inside = ((rec.member >> i) & 1).astype(bool)
        esc = ~inside
        while True:
            bad = (deps >= 0) & esc[np.where(deps >= 0, deps, 0)]
            new = esc | (bad.any(axis=1) & free)
            if np.array_equal(new, esc):
                break
            esc = new
        ok = ~esc & inside
        assert np.abs(Vs[i][ok] - Vg[ok]).max(initial=0.0) <= 1e-12
        closed_any |= ok
    assert closed_any.mean() > 0.02
    assert np.abs(Vbar - Vg).max() <= 0.1 * max(p.dx)


def test_coarse_problem_samples_axis_factors_per_axis():
    p = W.pursuit_evasion_problem(49, split=4, m_a=8, m_b=4)
    a = I.coarse_problem(p.with_(coarse_stride=4))
    b = I.coarse_problem(p.with_(coarse_n=(13, 13)))
    assert np.array_equal(a.speed, b.speed) and a.speed.shape == (13 * 13, 2)
    S = np.asarray(p.speed).reshape(49, 49, 2)[::4, ::4].reshape(-1, 2)
    assert np.array_equal(a.speed, S)
    # on a non-nested grid each factor is its own Q1 sample (x2 + 1 is linear: exact)
    c = I.coarse_problem(p.with_(coarse_n=(17, 17)))
    Xc = W.node_coords((17, 17), (-1.0, -1.0), (1.0, 1.0))
    assert np.abs(c.speed[:, 0] - (Xc[:, 1] + 1.0)).max() <= 1e-6
    assert np.array_equal(c.speed[:, 1], np.ones(17 * 17))
