"""Exact policy iteration (Howard's algorithm) for the SL scheme on tiny grids.

TEST INFRASTRUCTURE ONLY.  An independent way to reach the fixed point of the
scheme V = T(V) (paper Sec. 3, (SL)/(Tdef)): instead of iterating T, alternate
  * policy evaluation: solve the linear system V = beta P_pi V + w l (+ fixed and
    ghost contributions) exactly, in rational arithmetic, and
  * policy improvement: pi(j) = a minimiser of beta I[V](foot_k) + w l_j,
until the policy is stable.  The foot positions and the Q1 (or P1) weights are evaluated
exactly from the (binary64) problem data, so the only inexact inputs are the
binary64 values of beta and w.  Only practical for grids of a few dozen free
nodes.

For a differential game (paper Sec. 2; the evader's choice b_l is maximised,
the pursuer's control a_k minimised) the fixed point is the pointwise maximum over
the evader's stationary strategies sigma (a choice l per node) of the value of the
control problem that sigma leaves to the pursuer: for every sigma the game value
is a supersolution of that problem (T_sigma V <= T V = V, so its value is below),
and the maximising choices at the game value give a sigma whose value it is.
``game_value`` enumerates every sigma on a tiny grid and solves each control
problem by the exact policy iteration above.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr
from typing import List, Tuple

import numpy as np


def _consts(lam: float, h: float, disc: str) -> Tuple[Fr, Fr]:
    if disc == "kruzkov":
        raise ValueError("the Kruzkov form has a per-node discount: use _node_consts")
    if disc == "exp":
        beta = Fr(math.exp(-lam * h))
        return beta, (1 - beta) / Fr(lam)
    beta = 1 / (1 + Fr(lam) * Fr(h))
    return beta, Fr(h)


def _node_consts(prob):
    """Per free node (discount, cost term): the problem's constants times l_j, or for
    the Kruzkov form beta_j = exp(-h l_j) and 1 - beta_j, from the same binary64
    exponentials the scheme uses (math.exp, math.expm1)."""
    lv = [1.0] * prob.N if prob.cost is None else [float(x) for x in prob.cost]
    if prob.disc == "kruzkov":
        h = float(prob.step)
        return [(Fr(math.exp(-h * l)), Fr(-math.expm1(-h * l))) for l in lv]
    beta, w = _consts(prob.lam, prob.step, prob.disc)
    return [(beta, w * Fr(l)) for l in lv]


def _floor(x: Fr) -> int:
    return x.numerator // x.denominator


def _table(prob):
    """Rows of the control table: the pursuer's controls a_k, or for a game the
    differences a_k - b_l in the order l m + k (exact rationals)."""
    A = [[Fr(float(x)) for x in row] for row in np.asarray(prob.velocity)]
    vb = getattr(prob, "velocity_b", None)
    if vb is None:
        return A
    return [[a[d] - Fr(float(b[d])) for d in range(prob.dim)]
            for b in np.asarray(vb) for a in A]


def _kuhn_stencil(p, tau, n):
    """P1 on the Kuhn simplex holding the point p + tau: its vertices start at the
    cell's lower corner p and step one axis at a time, in the order of decreasing
    fraction; the barycentric weights of the point are 1 - t_0, t_0 - t_1, ..,
    t_{d-1} for the sorted fractions (exact rationals; a tie gives a zero weight,
    so its order does not matter)."""
    dim = len(p)
    order = sorted(range(dim), key=lambda d: -tau[d])
    t = [tau[d] for d in order]
    w = [1 - t[0]] + [t[i - 1] - t[i] for i in range(1, dim)] + [t[dim - 1]]
    v = list(p)
    st = []
    for i in range(dim + 1):
        if i > 0:
            v[order[i - 1]] += 1
        inside = all(0 <= v[d] < n[d] for d in range(dim))
        idx, stride = 0, 1
        for d in range(dim):
            idx += v[d] * stride
            stride *= n[d]
        if w[i] != 0:
            st.append((idx if inside else -1, w[i]))
    return st


def exact_stencils(prob):
    """For every free node and table row: list of (corner index or -1, weight)."""
    dim, n = prob.dim, prob.n
    N = prob.N
    h = Fr(prob.step)
    t = [h / ((Fr(prob.hi[d]) - Fr(prob.lo[d])) / (n[d] - 1)) for d in range(dim)]
    tgt = np.asarray(prob.target)
    rows = _table(prob)
    sp = None if prob.speed is None else np.asarray(prob.speed)
    out = {}
    for j in range(N):
        if tgt[j] >= 0:
            continue
        ij = []
        r = j
        for d in range(dim):
            ij.append(r % n[d])
            r //= n[d]
        if sp is None:
            c = [Fr(1)] * dim
        elif sp.ndim == 2:
            c = [Fr(float(sp[j, d])) for d in range(dim)]
        else:
            c = [Fr(float(sp[j]))] * dim
        q = [Fr(0)] * dim if prob.drift is None else \
            [t[d] * Fr(float(np.asarray(prob.drift).reshape(-1, dim)[j, d])) for d in range(dim)]
        per_k = []
        for row in rows:
            # foot x + h (b(x) + S(x) e) with e = a_k (or a_k - b_l), in index units
            u = [ij[d] + t[d] * row[d] * c[d] + q[d] for d in range(dim)]
            p = [_floor(x) for x in u]
            tau = [u[d] - p[d] for d in range(dim)]
            st = []
            if getattr(prob, "interp", "q1") == "p1":
                per_k.append(_kuhn_stencil(p, tau, n))
                continue
            for s in range(1 << dim):
                w = Fr(1)
                idx, stride, inside = 0, 1, True
                for d in range(dim):
                    bit = (s >> d) & 1
                    w *= tau[d] if bit else 1 - tau[d]
                    pd = p[d] + bit
                    if pd < 0 or pd >= n[d]:
                        inside = False
                    idx += pd * stride
                    stride *= n[d]
                if w != 0:
                    st.append((idx if inside else -1, w))
            per_k.append(st)
        out[j] = per_k
    return out


def _solve_exact(A: List[List[Fr]], b: List[Fr]) -> List[Fr]:
    """Gauss-Jordan elimination with exact fractions (A is diagonally dominant)."""
    n = len(b)
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        if piv != col:
            M[col], M[piv] = M[piv], M[col]
        inv = 1 / M[col][col]
        rowc = [x * inv for x in M[col]]
        M[col] = rowc
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [a - f * bb for a, bb in zip(M[r], rowc)]
    return [M[i][n] for i in range(n)]


def policy_iteration(prob, max_iter: int = 100, st=None, rows=None):
    """Exact fixed point of the scheme by Howard's algorithm (a control problem:
    the minimum over the table rows ``rows[j]`` a node may use, all rows when
    ``rows`` is None).

    Returns (V as a list of Fractions over all nodes, policy array, iterations)."""
    bw = _node_consts(prob)
    G = Fr(float(prob.v_ghost))
    tgt = np.asarray(prob.target)
    gv = [Fr(0)] * prob.N if prob.g is None else [Fr(float(x)) for x in prob.g]
    if st is None:
        st = exact_stencils(prob)
    free = sorted(st)
    if rows is None:
        if getattr(prob, "velocity_b", None) is not None:
            raise ValueError("a game needs game_value (or explicit rows)")
        rows = {j: range(prob.m) for j in free}
    pos = {j: i for i, j in enumerate(free)}
    fixedval = {j: gv[j] for j in range(prob.N) if tgt[j] >= 0}
    pol = {j: rows[j][0] for j in free}
    V = None
    for it in range(1, max_iter + 1):
        nf = len(free)
        A = [[Fr(0)] * nf for _ in range(nf)]
        b = [Fr(0)] * nf
        for j in free:
            r = pos[j]
            beta, wl = bw[j]
            A[r][r] += 1
            b[r] += wl
            for idx, wt in st[j][pol[j]]:
                if idx < 0:
                    b[r] += beta * wt * G
                elif idx in fixedval:
                    b[r] += beta * wt * fixedval[idx]
                else:
                    A[r][pos[idx]] -= beta * wt
        x = _solve_exact(A, b)
        V = [Fr(0)] * prob.N
        for j in range(prob.N):
            V[j] = fixedval.get(j, Fr(0))
        for j in free:
            V[j] = x[pos[j]]

        def val(j, k):
            acc = Fr(0)
            for idx, wt in st[j][k]:
                acc += wt * (G if idx < 0 else V[idx])
            return bw[j][0] * acc + bw[j][1]

        changed = False
        for j in free:
            cur = val(j, pol[j])
            best, bk = cur, pol[j]
            for k in rows[j]:
                v = val(j, k)
                if v < best:
                    best, bk = v, k
            if bk != pol[j]:
                pol[j] = bk
                changed = True
        if not changed:
            policy = np.full(prob.N, -1, dtype=np.int64)
            for j in free:
                policy[j] = pol[j]
            return V, policy, it
    raise RuntimeError("policy iteration did not converge")


def candidate_gaps(prob, V) -> np.ndarray:
    """Per free node: gap between the best and second-best control value at V
    (exact), to know where a policy comparison is meaningful."""
    beta, w = _consts(prob.lam, prob.step, prob.disc)
    G = Fr(float(prob.v_ghost))
    lv = [Fr(1)] * prob.N if prob.cost is None else [Fr(float(x)) for x in prob.cost]
    st = exact_stencils(prob)
    gaps = np.full(prob.N, np.inf)
    for j, per_k in st.items():
        vals = []
        for k in range(prob.m):
            acc = Fr(0)
            for idx, wt in per_k[k]:
                acc += wt * (G if idx < 0 else V[idx])
            vals.append(beta * acc + w * lv[j])
        vals.sort()
        gaps[j] = float(vals[1] - vals[0]) if len(vals) > 1 else np.inf
    return gaps


def game_value(prob, max_iter: int = 100):
    """Exact fixed point of the game scheme max_l min_k on a tiny grid: the
    pointwise maximum, over every stationary evader strategy sigma, of the exact
    value of the control problem sigma leaves to the pursuer (rows sigma(j) m + k).

    Returns (V as a list of Fractions, the number of strategies, and whether one
    strategy attains the maximum at every node)."""
    import itertools
    mb = np.asarray(prob.velocity_b).shape[0]
    m = prob.m
    st = exact_stencils(prob)
    free = sorted(st)
    best = None
    values = []
    for sigma in itertools.product(range(mb), repeat=len(free)):
        rows = {j: range(s * m, s * m + m) for j, s in zip(free, sigma)}
        V, _, _ = policy_iteration(prob, max_iter, st=st, rows=rows)
        best = V if best is None else [max(a, b) for a, b in zip(best, V)]
        values.append(V)
    attained = any(all(v == b for v, b in zip(V, best)) for V in values)
    return best, mb ** len(free), attained

