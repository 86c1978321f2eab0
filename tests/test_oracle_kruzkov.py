"""Pins of the oracle's Kruzkov form of the weighted minimum-time problem
(disc = "kruzkov": per node beta_j = exp(-h l_j), cost term 1 - beta_j, so that
v = 1 - exp(-J) with J the l-weighted time to the target; Sec. 2).  No GPU."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import tiny


def _line(n=41, n_y=5):
    """a in {+-e1, +-e2}, h = dx, target = the leftmost column, l varying with x1
    only: the optimal path runs left along its row and every foot is a node."""
    X = W.node_coords((n, n_y), (-1.0, -1.0), (1.0, 1.0))
    i0 = np.arange(X.shape[0]) % n
    l = W.f32(1.0 + 0.5 * np.sin(3.0 * X[:, 0]) ** 2)
    return W.Problem(name="kruzkov_line", dim=2, n=(n, n_y), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                     velocity=np.array([[-1.0, 0.0], [1.0, 0.0], [0.0, 1.0], [0.0, -1.0]]),
                     target=np.where(i0 == 0, 0, -1).astype(np.int8), n_comp=1, cost=l,
                     v_ghost=2.0, disc="kruzkov"), i0, l


def test_line_closed_form_is_one_minus_exp_of_the_weighted_time():
    """1 - V_i = prod_{k=1..i} exp(-h l_k) = exp(-h sum l_k): the Kruzkov image of
    the left Riemann sum of the weighted time."""
    p, i0, l = _line()
    V, _, _, _ = O.solve(p)
    h = p.step
    lcol = l.reshape(p.n[1], p.n[0])[0]
    J = np.concatenate([[0.0], np.cumsum(h * lcol[1:])])
    want = 1.0 - np.exp(-J[i0])
    assert np.abs(V - want).max() <= 1e-14
    # the discounted form with a constant rate instead would not match
    assert np.abs(O.solve(p.with_(disc="exp"))[0] - want).max() > 1e-3


def test_constant_cost_equals_the_discounted_form():
    """l = c0 everywhere: beta = exp(-h c0) and 1 - beta, the discounted scheme with
    lam = c0 and running cost c0 (equal up to the rounding of w l)."""
    base = W.c2_multitarget(n=65, m=16)
    c0 = 1.75
    p = base.with_(speed=None, cost=np.full(base.N, c0), v_ghost=2.0)
    Vk, _, _, _ = O.solve(p.with_(disc="kruzkov"))
    Ve, _, _, _ = O.solve(p.with_(disc="exp", lam=c0))
    assert np.abs(Vk - Ve).max() <= 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_exact_policy_iteration(dim):
    if dim == 2:
        p = W.kruzkov_problem(n=7, m=8, n_disks=1, r=0.3)
    else:
        base = W.c3_aniso3d(n=4, m=10, n_balls=1, r=0.5)
        X = W.node_coords(base.n, base.lo, base.hi)
        p = base.with_(speed=None, cost=W.f32(1.0 + 0.4 * X[:, 0] ** 2), v_ghost=2.0,
                       disc="kruzkov")
    Vx, pol, it = tiny.policy_iteration(p)
    V, _, _, _ = O.solve(p)
    assert np.abs(V - np.array([float(x) for x in Vx])).max() <= 1e-13


def test_ghost_two_is_a_supersolution_in_floating_point():
    """T(V0) <= V0 exactly for V0 = v_ghost = 2 on free nodes (the premise of the
    order-independence of the iteration)."""
    p = W.kruzkov_problem(n=65, m=16)
    V0 = O.initial_values(p)
    TV, _ = O.apply_T(p, V0)
    assert (TV <= V0).all()
