"""Brute-force pins of the FP64 oracle on tiny inputs (no GPU)."""
import itertools

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import isa as I
from oracle import tiny


def _tiny_2d(n, m, seed, disc="exp", cost=False, ghost=1.0):
    p = W.c2_multitarget(n=n, m=m, n_disks=2, r=0.05, seed_field=seed, seed_disks=seed + 1)
    if cost:
        rng = np.random.Generator(np.random.PCG64(seed + 7))
        p = p.with_(cost=W.f32(np.exp(rng.normal(0, 0.3, p.N))), v_ghost=ghost)
    return p.with_(disc=disc)


CASES = [
    ("2d_n7_m8", lambda: _tiny_2d(7, 8, 11)),
    ("2d_n9_m8", lambda: _tiny_2d(9, 8, 21)),
    ("2d_n11_m16", lambda: _tiny_2d(11, 16, 31)),
    ("2d_cost_ghost2", lambda: _tiny_2d(9, 8, 41, cost=True, ghost=3.0)),
    ("2d_paper_disc", lambda: _tiny_2d(9, 8, 51, disc="paper")),
    ("2d_m7_odd", lambda: _tiny_2d(9, 7, 61)),
    ("3d_n4_m10", lambda: W.c3_aniso3d(n=4, m=10, n_balls=1, r=0.5)),
    # control-affine dynamics with a drift (Van der Pol, Sec. 4.1): f = b(x) + (0, a)
    ("2d_vdp_drift_n9", lambda: W.vdp_problem(9, split=1, n_a=5)),
    ("2d_vdp_drift_n11_split2", lambda: W.vdp_problem(11, split=2, n_a=7, rho=0.25)),
]


@pytest.mark.parametrize("name,mk", CASES, ids=[c[0] for c in CASES])
def test_jacobi_matches_exact_policy_iteration(name, mk):
    """The oracle's Jacobi fixed point (paper Sec. 3: V^{n+1} = T(V^n)) equals the
    exact fixed point found by Howard's policy iteration with rational linear
    solves, and the policies agree wherever the best control is not tied."""
    p = mk()
    Vx, pol_x, _ = tiny.policy_iteration(p)
    V, pol, _, res = O.solve(p)
    assert res == 0.0
    Vf = np.array([float(v) for v in Vx])
    assert np.abs(Vf - V).max() <= 1e-13
    gaps = tiny.candidate_gaps(p, Vx)
    clear = (pol_x >= 0) & (gaps > 1e-12)
    assert (pol[clear] == pol_x[clear]).all()


def _con_bruteforce(member_K, nK, n):
    """Con(.) by geometry: fine node j of an axis lies at coarse coordinate
    j (nK-1)/(n-1) (both grids span the same box); it is in set i iff a closed
    coarse cell containing it has all corners in set i; orphans take every set at
    the corners of the cells containing them.  Containment is tested exactly in
    integers: base (n-1) <= j (nK-1) <= (base+1) (n-1)."""
    dim = len(n)
    mK = member_K.reshape(tuple(reversed(nK)))

    def kval(idx):            # idx in x, y, (z) order
        return int(mK[tuple(reversed(idx))])

    out = np.zeros(tuple(reversed(n)), dtype=np.uint8)
    for fine in itertools.product(*[range(n[d]) for d in range(dim)]):
        cells = []
        for base in itertools.product(*[range(nK[d] - 1) for d in range(dim)]):
            if all(base[d] * (n[d] - 1) <= fine[d] * (nK[d] - 1) <= (base[d] + 1) * (n[d] - 1)
                   for d in range(dim)):
                cells.append(base)
        full = 0
        anyb = 0
        for base in cells:
            corners = [kval(tuple(base[d] + ((c >> d) & 1) for d in range(dim)))
                       for c in range(1 << dim)]
            a = 0xFF
            for v in corners:
                a &= v
                anyb |= v
            full |= a
        out[tuple(reversed(fine))] = full if full else anyb
    return out.reshape(-1)


@pytest.mark.parametrize("dim,nK,n,seed", [
    (2, (5, 4), (13, 10), 1), (2, (6, 6), (11, 11), 2), (3, (3, 4, 3), (5, 7, 5), 3),
    (2, (4, 4), (4, 4), 4),
    # coarse grids not nested in the fine grid
    (2, (5, 4), (12, 11), 5), (2, (7, 3), (10, 8), 6), (3, (3, 4, 4), (7, 6, 9), 7),
    (2, (15, 15), (41, 41), 8)])
def test_projection_matches_geometric_bruteforce(dim, nK, n, seed):
    """ISA step 2 (Sec. 4, Con(.) = union of the cells with all vertices in the set)
    against a geometric brute force on random coarse bitmasks."""
    from fractions import Fraction
    rng = np.random.Generator(np.random.PCG64(seed))
    NK = int(np.prod(nK))
    # random sets with some structure: a few bits set with high probability
    member_K = (rng.random((NK, 3)) < np.array([0.7, 0.5, 0.3])).astype(np.uint8)
    member_K = (member_K[:, 0] | (member_K[:, 1] << 1) | (member_K[:, 2] << 2)).astype(np.uint8)
    label_K = rng.integers(0, 3, NK).astype(np.uint8)
    mem, lab = I.project(member_K, label_K, nK, n)
    assert (mem == _con_bruteforce(member_K, nK, n)).all()
    # nearest coarse node label (ties rounded up), by exact rational rounding
    lk = label_K.reshape(tuple(reversed(nK)))
    for j in range(int(np.prod(n))):
        idx, r = [], j
        for d in range(dim):
            idx.append(r % n[d])
            r //= n[d]
        near = [min(int(Fraction(idx[d] * (nK[d] - 1), n[d] - 1) + Fraction(1, 2)), nK[d] - 1)
                for d in range(dim)]
        assert lab[j] == lk[tuple(reversed(near))]
