"""Exact policy iteration (Howard's algorithm) for the SL scheme on tiny grids.

TEST INFRASTRUCTURE ONLY.  An independent way to reach the fixed point of the
scheme V = T(V) (paper Sec. 3, (SL)/(Tdef)): instead of iterating T, alternate
  * policy evaluation: solve the linear system V = beta P_pi V + w l (+ fixed and
    ghost contributions) exactly, in rational arithmetic, and
  * policy improvement: pi(j) = a minimiser of beta I[V](foot_k) + w l_j,
until the policy is stable.  The foot positions and Q1 weights are evaluated
exactly from the (binary64) problem data, so the only inexact inputs are the
binary64 values of beta and w.  Only practical for grids of a few dozen free
nodes.
"""
from __future__ import annotations

import math
from fractions import Fraction as Fr
from typing import List, Tuple

import numpy as np


def _consts(lam: float, h: float, disc: str) -> Tuple[Fr, Fr]:
    if disc == "exp":
        beta = Fr(math.exp(-lam * h))
        return beta, (1 - beta) / Fr(lam)
    beta = 1 / (1 + Fr(lam) * Fr(h))
    return beta, Fr(h)


def _floor(x: Fr) -> int:
    return x.numerator // x.denominator


def exact_stencils(prob):
    """For every free node and control: list of (corner index or -1, weight)."""
    dim, n = prob.dim, prob.n
    N = prob.N
    h = Fr(prob.step)
    t = [h / ((Fr(prob.hi[d]) - Fr(prob.lo[d])) / (n[d] - 1)) for d in range(dim)]
    tgt = np.asarray(prob.target)
    out = {}
    for j in range(N):
        if tgt[j] >= 0:
            continue
        ij = []
        r = j
        for d in range(dim):
            ij.append(r % n[d])
            r //= n[d]
        c = Fr(1) if prob.speed is None else Fr(float(prob.speed[j]))
        q = [Fr(0)] * dim if prob.drift is None else \
            [t[d] * Fr(float(np.asarray(prob.drift).reshape(-1, dim)[j, d])) for d in range(dim)]
        per_k = []
        for k in range(prob.m):
            # foot x + h (b(x) + c(x) a_k), in index units
            u = [ij[d] + t[d] * Fr(float(prob.velocity[k, d])) * c + q[d] for d in range(dim)]
            p = [_floor(x) for x in u]
            tau = [u[d] - p[d] for d in range(dim)]
            st = []
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


def policy_iteration(prob, max_iter: int = 100):
    """Exact fixed point of the scheme by Howard's algorithm.

    Returns (V as a list of Fractions over all nodes, policy array, iterations)."""
    beta, w = _consts(prob.lam, prob.step, prob.disc)
    G = Fr(float(prob.v_ghost))
    tgt = np.asarray(prob.target)
    gv = [Fr(0)] * prob.N if prob.g is None else [Fr(float(x)) for x in prob.g]
    lv = [Fr(1)] * prob.N if prob.cost is None else [Fr(float(x)) for x in prob.cost]
    st = exact_stencils(prob)
    free = sorted(st)
    pos = {j: i for i, j in enumerate(free)}
    fixedval = {j: gv[j] for j in range(prob.N) if tgt[j] >= 0}
    pol = {j: 0 for j in free}
    V = None
    for it in range(1, max_iter + 1):
        nf = len(free)
        A = [[Fr(0)] * nf for _ in range(nf)]
        b = [Fr(0)] * nf
        for j in free:
            r = pos[j]
            A[r][r] += 1
            b[r] += w * lv[j]
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
            return beta * acc + w * lv[j]

        changed = False
        for j in free:
            cur = val(j, pol[j])
            best, bk = cur, pol[j]
            for k in range(prob.m):
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
