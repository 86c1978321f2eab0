"""Pins of the oracle's recursive refinement of the target split (the balance
remedy of the paper's conclusions, Sec. 5): the halving rule on shapes whose
answer is known, its partition invariants, and refinement runs.  No GPU."""
import numpy as np
import pytest

import workloads as W
from oracle import isa as I


def _grid_ids(n, pts):
    return [i + n[0] * j for i, j in pts]


def test_horizontal_segment_splits_into_left_and_right_halves():
    n = (16, 11)
    tid = np.full(n[0] * n[1], -1, np.int8)
    seg = _grid_ids(n, [(i, 5) for i in range(3, 13)])     # x extent 9, y extent 0
    tid[seg] = 2
    out = I.split_component(tid, n, 2, 5)
    assert list(out[seg]) == [2] * 5 + [5] * 5
    assert (out[np.setdiff1d(np.arange(tid.size), seg)] == -1).all()


def test_vertical_segment_odd_count_moves_the_upper_floor_half():
    n = (9, 12)
    tid = np.full(n[0] * n[1], -1, np.int8)
    seg = _grid_ids(n, [(4, j) for j in range(2, 9)])      # 7 nodes along y
    tid[seg] = 0
    out = I.split_component(tid, n, 0, 1)
    assert list(out[seg]) == [0, 0, 0, 0, 1, 1, 1]


def test_equal_extents_take_the_lowest_axis_and_break_ties_by_flat_index():
    n = (10, 10)
    tid = np.full(100, -1, np.int8)
    block = _grid_ids(n, [(i, j) for j in (3, 4) for i in (5, 6)])   # 2x2 block
    tid[block] = 0
    out = I.split_component(tid, n, 0, 1)
    # axis 0 (x): order (x=5, y=3), (x=5, y=4), (x=6, y=3), (x=6, y=4)
    assert out[5 + 10 * 3] == 0 and out[5 + 10 * 4] == 0
    assert out[6 + 10 * 3] == 1 and out[6 + 10 * 4] == 1


@pytest.mark.parametrize("seed,dim", [(1, 2), (2, 2), (3, 3)])
def test_halving_is_a_partition_ordered_along_the_axis(seed, dim):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = (13, 9) if dim == 2 else (7, 6, 5)
    N = int(np.prod(n))
    tid = np.where(rng.random(N) < 0.3, rng.integers(0, 3, N), -1).astype(np.int8)
    before = np.flatnonzero(tid == 1)
    out = I.split_component(tid, n, 1, 3)
    kept, moved = np.flatnonzero(out == 1), np.flatnonzero(out == 3)
    assert np.array_equal(np.union1d(kept, moved), before)
    assert len(moved) == len(before) // 2
    assert np.array_equal(out[out != 3], tid[out != 3])
    idx = np.stack(np.unravel_index(before, tuple(reversed(n)))[::-1], axis=1)
    axis = int(np.argmax(idx.max(0) - idx.min(0)))
    coord = lambda j: (j // int(np.prod(n[:axis]))) % n[axis]
    assert coord(kept).max() <= coord(moved).min()


def test_refinement_of_the_box_boundary():
    """Distance to the box boundary, Gamma = the whole boundary as one component:
    the single set is the whole box, and three halvings give four components whose
    largest set is under half of the box."""
    p = W.box_distance_problem(65, split=1).with_(coarse_stride=4)
    tid, nc, hist = I.refine_split(p, 4)
    assert nc == 4 and len(hist) == 4
    assert hist[0] == 1.0 and hist[-1] < 0.5
    assert sorted(np.unique(tid[tid >= 0])) == [0, 1, 2, 3]
    assert np.array_equal(tid >= 0, np.asarray(p.target) >= 0)


def test_refinement_stops_at_the_goal():
    p = W.box_distance_problem(65, split=1).with_(coarse_stride=4)
    tid, nc, hist = I.refine_split(p, 8, frac_goal=0.7)
    assert hist[-1] <= 0.7 and all(h > 0.7 for h in hist[:-1])
    assert nc == len(hist)
