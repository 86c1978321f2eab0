"""Pins of the FP64 oracle against closed forms fixed by the paper and by the
mathematics of the scheme (no GPU)."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import isa as I


def _cells_to_nearest_line(n):
    i0 = np.arange(n)
    return np.minimum(i0, n - 1 - i0)


@pytest.mark.parametrize("n", [21, 41])
@pytest.mark.parametrize("delta", [1.0, 0.1])
def test_strip_exact(n, delta):
    """Strip example (Sec. 3, Example 3.1; closed form corrected so that v = 0 on
    x1 = +-1): v(x) = (1 - exp(-delta (1 - |x1|)))/delta.  With h = dx the axis
    control's foot lands on a node and every other foot is no better, so the
    discrete solution equals the closed form at every node."""
    p = W.strip_problem(n, delta)
    V, pol, s, res = O.solve(p)
    assert res == 0.0
    k = _cells_to_nearest_line(n)
    X = W.grid_axes(p.n, p.lo, p.hi)[0]
    exact = (1.0 - np.exp(-delta * (1.0 - np.abs(X)))) / delta
    Vg = V.reshape(n, n)
    assert np.abs(Vg - exact[None, :]).max() <= 1e-13
    # x2-invariance: every row is the same
    assert np.abs(Vg - Vg[n // 2][None, :]).max() <= 1e-15
    # geometric-sum form of the discrete recurrence V(k) = beta V(k-1) + w
    beta, w = O.scheme_constants(delta, p.step, "exp")
    geo = np.array([w * sum(beta ** i for i in range(kk)) for kk in k])
    assert np.abs(Vg[n // 2] - geo).max() <= 1e-13


def test_strip_paper_discount():
    """Same strip with the discount printed in (Tdef): beta = 1/(1+lam h), w = h.
    The discrete value at k cells is the geometric sum h (1 + beta + ... + beta^(k-1))."""
    n, delta = 31, 1.0
    p = W.strip_problem(n, delta).with_(disc="paper")
    V, _, _, res = O.solve(p)
    assert res == 0.0
    beta, w = O.scheme_constants(delta, p.step, "paper")
    assert beta == 1.0 / (1.0 + delta * p.step) and w == p.step
    k = _cells_to_nearest_line(n)
    geo = np.array([w * sum(beta ** i for i in range(kk)) for kk in k])
    assert np.abs(V.reshape(n, n)[n // 2] - geo).max() <= 1e-13


@pytest.mark.parametrize("n", [41, 101])
def test_point_target_axes_and_lower_bound(n):
    """Point target, f = a, |a| = 1: on the axes through the target the discrete
    value is 1 - beta^k (k cells away); everywhere it is >= 1 - beta^(Chebyshev
    distance), since one step moves the foot by at most one cell per axis."""
    p = W.c1_eikonal(n)
    V, _, _, res = O.solve(p)
    assert res == 0.0
    beta, _ = O.scheme_constants(1.0, p.step)
    c = n // 2
    Vg = V.reshape(n, n)
    k = np.abs(np.arange(n) - c)
    assert np.abs(Vg[c, :] - (1.0 - beta ** k)).max() <= 1e-14
    assert np.abs(Vg[:, c] - (1.0 - beta ** k)).max() <= 1e-14
    # equals the continuous Kruzkov distance 1 - exp(-|x|) there
    assert np.abs(Vg[c, :] - (1.0 - np.exp(-k * p.dx[0]))).max() <= 1e-14
    cheb = np.maximum(k[:, None], k[None, :])
    assert (Vg - (1.0 - beta ** cheb)).min() >= -1e-14   # ~k ulps of rounding
    assert V.max() <= p.v_ghost and V.min() >= 0.0


def test_point_target_converges_to_closed_form():
    """V -> 1 - exp(-|x|) (the Kruzkov transform of the distance) as the grid is
    refined with h = dx (Theorem 3.1): the sup error decreases and is O(1e-2)."""
    errs = []
    for n in (51, 101, 201):
        p = W.c1_eikonal(n)
        V, _, _, _ = O.solve(p)
        X = W.node_coords(p.n, p.lo, p.hi)
        ex = 1.0 - np.exp(-np.hypot(X[:, 0], X[:, 1]))
        errs.append(np.abs(V - ex).max())
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] < 1e-2
    # roughly first order in dx
    assert errs[1] / errs[2] > 1.5


@pytest.mark.parametrize("split", [1, 4])
def test_box_distance_exact(split):
    """Distance to the boundary of (-1,1)^2 with lambda = 1 (Sec. 4.1, first
    example; closed form with max, not min, so that v = 0 on the boundary):
    v = 1 - exp(-(1 - max|x_i|)).  The discrete solution equals it at the nodes
    (axis control to the nearest edge; Chebyshev lower bound)."""
    n = 41
    p = W.box_distance_problem(n, split=split)
    V, _, _, res = O.solve(p)
    assert res == 0.0
    X = W.node_coords(p.n, p.lo, p.hi)
    ex = 1.0 - np.exp(-(1.0 - np.maximum(np.abs(X[:, 0]), np.abs(X[:, 1]))))
    assert np.abs(V - ex).max() <= 1e-14


def test_box_distance_isa_triangles():
    """4-way split of the boundary: the exact independent sub-domains are the
    four triangles (25% each, Table 1 last column).  The reconstructed sets
    contain them and the ISA reproduces the global solution."""
    n = 81
    p = W.box_distance_problem(n, split=4).with_(coarse_stride=4, ra_C=0.25, ra_M=0.25)
    Vg, _, _, _ = O.solve(p)
    Vbar, owner, rec, Vs, _ = I.isa(p)
    assert np.abs(Vbar - Vg).max() <= 1e-14
    X = W.node_coords(p.n, p.lo, p.hi)
    x1, x2 = X[:, 0], X[:, 1]
    # component ids: 0 bottom (x2=-1), 1 right, 2 top, 3 left
    dist = np.stack([1 + x2, 1 - x1, 1 - x2, 1 + x1], axis=1)
    dmin = dist.min(axis=1)
    for i in range(4):
        true_set = dist[:, i] <= dmin + 1e-12
        bit = ((rec.member >> i) & 1).astype(bool)
        assert bit[true_set].all(), f"true sub-domain {i} not contained"
    frac = max(((rec.member >> i) & 1).mean() for i in range(4))
    assert 0.25 <= frac <= 0.35


def test_box_distance_ra_matches_table1():
    """Table 1 (Sec. 4.1): max_i |Sigma_i| / |Omega| of the RA on coarse grids with
    dx_K = 2/N, 4-way split.  With the threshold delta = dx_K the oracle's RA
    reproduces every printed fraction to within 3 percentage points, and the
    fractions shrink towards the exact 25% as the grid is refined."""
    import json, os
    T = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "paper_tables.json")))["distance_function_ra"]
    ours = []
    for N, ref in zip(T["N_side"], T["max_set_fraction"]):
        p = W.box_distance_problem(N + 1, split=4).with_(ra_C=0.25, ra_M=0.25)
        mK, _, _, _, delta, _ = I.reconstruct_on(p)
        assert abs(delta - 2.0 / N) < 1e-15
        fr = max(((mK >> i) & 1).mean() for i in range(4))
        assert abs(fr - ref) <= 0.03, (N, fr, ref)
        ours.append(fr)
    assert all(a >= b for a, b in zip(ours, ours[1:]))
    assert ours[-1] > T["exact_max_set_fraction"]


@pytest.mark.parametrize("n", [41, 81])
def test_constant_drift_exact(n):
    """Control-affine dynamics f = b + a with a constant drift b = (1, 0) and unit
    controls, target on the right edge only, h = dx/2: the best control a = e1
    moves exactly one cell per step (drift and control each half a cell), every
    other control progresses less towards the target, so the scheme is exact at
    the nodes: V = 1 - exp(-(1 - x1)/2) (travel time (1 - x1)/2 at speed 2).
    A dropped or mis-signed drift term changes the travel time."""
    p = W.strip_problem(n, 1.0)
    tid = np.full(p.N, -1, dtype=np.int8)
    tid.reshape(n, n)[:, -1] = 0
    dx = 2.0 / (n - 1)
    drift = np.zeros((p.N, 2))
    drift[:, 0] = 1.0
    q = p.with_(target=tid, n_comp=1, drift=drift, h=dx / 2, v_ghost=1.0)
    V, _, _, res = O.solve(q)
    assert res == 0.0
    X = W.node_coords(q.n, q.lo, q.hi)
    ex = 1.0 - np.exp(-(1.0 - X[:, 0]) / 2.0)
    assert np.abs(V - ex).max() <= 1e-13
