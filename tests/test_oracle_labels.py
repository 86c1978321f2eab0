"""Pins of the oracle's reconstruction label (RA step 3 of Sec. 3): the label of a
coarse node is the component whose auxiliary value is smallest there, the lowest
index on ties.  By Proposition 2.1 the exact sub-domain of component i is where
its auxiliary value equals the global one, so away from the interfaces the label
must name the component whose target the optimal trajectory reaches: for unit
speed, the nearest one.  Each test states that geometric fact independently of
the oracle's arithmetic, so a wrong rule (argmax, highest index on ties, the
label taken from another array) fails at least one of them."""
import numpy as np
import pytest

import workloads as W
from oracle import isa as I


def _ra_on(p):
    """RA steps 1-3 with the problem's own grid as the coarse grid K."""
    mK, lK, V_aux, V, delta, _ = I.reconstruct_on(p)
    return mK, lK, V_aux


@pytest.mark.parametrize("n", [33, 41])
def test_box_distance_label_is_the_nearest_edge_with_the_lowest_index_on_ties(n):
    """Distance to the boundary of the square split into its four edges (bottom 0,
    right 1, top 2, left 3; Sec. 4.1's 4-way split).  The auxiliary value of edge i
    is 1 - exp(-k_i dx) with k_i the node's cell count to that edge (the axis
    control lands on nodes, so the scheme is exact there), hence the label is the
    nearest edge at every free node.  On the diagonals two edges are equally near,
    their auxiliary values are equal bit for bit, and the lower index must win."""
    p = W.box_distance_problem(n, split=4)
    mK, lK, V_aux = _ra_on(p)
    j = np.arange(p.N)
    i0, i1 = j % n, j // n
    cells = np.stack([i1, n - 1 - i0, n - 1 - i1, i0])        # to bottom, right, top, left
    free = np.asarray(p.target) < 0
    srt = np.sort(cells, axis=0)
    nearest = np.argmin(cells, axis=0)                          # lowest index on ties
    clear = free & (srt[1] > srt[0])
    tie = free & (srt[1] == srt[0])
    assert clear.sum() > 0.9 * free.sum() - 2 * n and tie.sum() >= n - 4
    assert np.array_equal(lK[clear], nearest[clear])
    # the tie is exact in the values, so the tie rule decides the label
    Va = np.stack(V_aux)
    for jj in np.flatnonzero(tie):
        tied = np.flatnonzero(cells[:, jj] == srt[0, jj])
        assert len(tied) >= 2
        assert np.all(Va[tied, jj] == Va[tied[0], jj])
        assert lK[jj] == tied.min()
    # aux values of the nearest edge: the closed form at the nodes
    dx = p.dx[0]
    exact = 1.0 - np.exp(-cells[nearest[free], np.flatnonzero(free)] * dx)
    assert np.abs(Va[nearest[free], np.flatnonzero(free)] - exact).max() <= 1e-13


def test_target_nodes_carry_their_own_component():
    """On a target node of component i the auxiliary value i is g = 0 and every
    other auxiliary problem reads the ghost value there, so the label is i."""
    p = W.c2_multitarget(n=65, m=32).with_(coarse_stride=1)
    _, lK, _ = _ra_on(p)
    tid = np.asarray(p.target)
    on = tid >= 0
    assert on.sum() >= p.n_comp
    assert np.array_equal(lK[on], tid[on].astype(np.uint8))


@pytest.mark.parametrize("dim", [2, 3])
def test_equal_disks_with_unit_speed_label_the_nearest_centre(dim):
    """Equal target disks (balls) and unit speed: the exact partition is the
    Voronoi diagram of the centres (the optimal trajectory runs straight to the
    nearest disk).  Wherever the nearest centre is closer than the second by more
    than 2 dx, the label must be that centre's component."""
    if dim == 2:
        n, m = 65, 32
        cen = np.array([[-0.5, -0.4], [0.45, -0.35], [0.05, 0.55]])
        vel = W.controls_2d(m)
        r = 0.08
    else:
        n, m = 21, 64
        cen = np.array([[-0.45, -0.4, -0.3], [0.5, -0.3, 0.2], [0.0, 0.5, -0.1]])
        vel = W.controls_3d_fibonacci(m)
        r = 0.12
    shape = (n,) * dim
    lo, hi = (-1.0,) * dim, (1.0,) * dim
    X = W.node_coords(shape, lo, hi)
    tid = W.ball_targets(shape, lo, hi, cen, r)
    p = W.Problem(name=f"voronoi{dim}", dim=dim, n=shape, lo=lo, hi=hi, velocity=vel,
                  target=tid, n_comp=len(cen), v_ghost=1.0, coarse_stride=1)
    _, lK, _ = _ra_on(p)
    dist = np.stack([np.sqrt(((X - c[None, :]) ** 2).sum(axis=1)) for c in cen])
    srt = np.sort(dist, axis=0)
    nearest = np.argmin(dist, axis=0)
    free = tid < 0
    clear = free & (srt[1] - srt[0] > 2.0 * p.dx[0])
    assert clear.sum() > 0.6 * free.sum()
    assert np.array_equal(lK[clear], nearest[clear].astype(np.uint8))


def test_a_node_no_target_reaches_is_labelled_zero():
    """Nodes of zero speed cannot move: every auxiliary problem computes the same
    value there from the same data (the ghost value, unchanged), so all
    components tie and the lowest index, 0, is the label."""
    n = 65
    p = W.c2_multitarget(n=n, m=32).with_(coarse_stride=1)
    X = W.node_coords((n, n), (-1.0, -1.0), (1.0, 1.0))
    sp = np.asarray(p.speed).copy()
    still = (np.abs(X[:, 0] - 0.9) < 0.08) & (np.abs(X[:, 1] + 0.9) < 0.08)
    still &= np.asarray(p.target) < 0
    sp[still] = 0.0
    q = p.with_(speed=sp)
    _, lK, V_aux = _ra_on(q)
    assert still.sum() >= 9
    Va = np.stack(V_aux)[:, still]
    assert np.all(Va == Va[0:1, :])
    assert np.all(lK[still] == 0)
