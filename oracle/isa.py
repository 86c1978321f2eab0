"""Reconstruction algorithm (RA, paper Sec. 3) and independent-sets algorithm (ISA,
paper Sec. 4), step by step as the paper lists them, on top of the FP64 SL solver.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Readings of the paper used here:
  * the coarse grid K is a second uniform grid on the same box (Sec. 4 lets the
    two triangulations differ; only both must cover the domain): nK_d nodes per
    axis (``prob.coarse_n``, or every s-th fine node for a stride s dividing
    n_d - 1).  Coarse node k of an axis lies at fine coordinate
    k (n_d - 1)/(nK_d - 1).  K takes speed, cost and drift by the scheme's own
    Q1 interpolation of the fine fields there (exact copies at coincident nodes),
    target id and exit cost g from the nearest fine node (ties rounded up); a
    component with no coarse node gets the coarse node nearest its lowest-index
    fine node; the SL step on K is h times the largest ratio
    (n_d - 1)/(nK_d - 1);
  * the auxiliary problem i (RA step 1, "T_i with boundary X_i") keeps component i
    at g and holds every other component's target nodes at the ghost value, a
    boundary datum larger than g ((gcond));
  * RA step 2: the (H2) check is skipped (a control problem's Hamiltonian is
    convex, Remark 2.1; for a game the caller vouches for the decomposability
    condition (C), as the paper shows for its pursuit-evasion example), then
    V = min_i V_i;
  * RA step 3 threshold delta = 2 (C dx^q + M dx) (Proposition 3.1), dx the coarse
    grid spacing (largest over axes);
  * ISA step 2, Con(.): a fine node belongs to the projected set iff some closed
    coarse cell containing it has all 2^d corners in the coarse set; a fine node
    left in no set receives every set present at a corner of its cells (so the
    sets cover the grid);
  * labels: the coarse argmin of V_i (lowest index on ties), pulled to the fine
    grid from the nearest coarse node (ties rounded up);
  * ISA step 3 solves T on each projected set, non-members reading the ghost value;
    ISA step 4 takes the minimum over the sets containing each node (owner = the
    lowest minimising index).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from . import initial_values, fixed_mask, solve


@dataclass
class Reconstruction:
    member_K: np.ndarray      # uint8 bitmask on K
    label_K: np.ndarray       # uint8 argmin label on K
    V_aux: List[np.ndarray]   # auxiliary values V_i on K
    V_K: np.ndarray           # min_i V_i on K
    delta: float
    nK: tuple
    member: np.ndarray        # uint8 bitmask on the fine grid (after projection)
    label: np.ndarray         # uint8 label on the fine grid
    sweeps: List[int]


def coarse_nodes(prob) -> tuple:
    """Nodes per axis of the coarse grid K: ``prob.coarse_n`` when given, else every
    s-th fine node (s = ``prob.coarse_stride`` must divide n_d - 1)."""
    if getattr(prob, "coarse_n", None):
        nK = tuple(int(k) for k in prob.coarse_n[:prob.dim])
        for d in range(prob.dim):
            if not 3 <= nK[d] <= prob.n[d]:
                raise ValueError("coarse node counts must lie in [3, n_d]")
        return nK
    s = int(prob.coarse_stride)
    for d in range(prob.dim):
        if (prob.n[d] - 1) % s:
            raise ValueError("coarse stride must divide n-1 on every axis")
    return tuple((prob.n[d] - 1) // s + 1 for d in range(prob.dim))


def fine_coordinate_of_coarse(n: int, nK: int):
    """Coarse node k of an axis sits at fine coordinate k (n-1)/(nK-1) = i0 + t with
    integer i0 and t = r/(nK-1) in [0, 1).  Returns (i0, i1 = min(i0+1, n-1), t, the
    nearest fine index with ties rounded up), all by integer arithmetic but t."""
    k = np.arange(nK, dtype=np.int64)
    P = k * (n - 1)
    i0 = P // (nK - 1)
    r = P % (nK - 1)
    t = r.astype(np.float64) / float(nK - 1)
    i1 = np.minimum(i0 + 1, n - 1)
    near = i0 + (2 * r >= nK - 1)
    return i0, i1, t, near


def coarse_coordinate_of_fine(n: int, nK: int):
    """Fine node j of an axis sits at coarse coordinate j (nK-1)/(n-1) = c + r/(n-1).
    Returns (c, r) as integers."""
    j = np.arange(n, dtype=np.int64)
    P = j * (nK - 1)
    return P // (n - 1), P % (n - 1)


def sample_q1(field: np.ndarray, n: tuple, nK: tuple) -> np.ndarray:
    """Q1 (multilinear) interpolation of a fine node field at the coarse nodes, in
    FP64: corner weights are products over the axes in axis order, and the corner
    terms are summed in corner order starting from 0 (corner bit d = upper node on
    axis d).  A coarse node that coincides with a fine node gets its value exactly."""
    dim = len(n)
    F = np.asarray(field, dtype=np.float64).reshape(tuple(reversed(n)))
    maps = [fine_coordinate_of_coarse(n[d], nK[d]) for d in range(dim)]
    acc = np.zeros(tuple(reversed(nK)))
    for corner in range(1 << dim):
        w = None
        idx = []
        for d in range(dim):
            i0, i1, t, _ = maps[d]
            up = (corner >> d) & 1
            wd = t if up else (1.0 - t)
            shape = [1] * dim
            shape[dim - 1 - d] = nK[d]            # numpy axis of grid axis d
            wd = wd.reshape(shape)
            w = wd if w is None else w * wd
            idx.append(i1 if up else i0)
        acc = acc + w * F[np.ix_(*reversed(idx))]
    return acc.reshape(-1)


def coarse_problem(prob):
    """The coarse grid K and its problem data (see the module notes)."""
    dim = prob.dim
    nK = coarse_nodes(prob)
    n = tuple(prob.n[:dim])
    shp = prob.shape()
    near = [fine_coordinate_of_coarse(n[d], nK[d])[3] for d in range(dim)]
    nearest_ix = np.ix_(*reversed(near))

    def nearest(a):
        return None if a is None else np.ascontiguousarray(
            np.asarray(a).reshape(shp)[nearest_ix]).reshape(-1)

    def q1(a):
        return None if a is None else sample_q1(a, n, nK)

    tid = nearest(prob.target).copy()
    g = nearest(prob.g)
    ftid = np.asarray(prob.target)
    cmap = [coarse_coordinate_of_fine(n[d], nK[d]) for d in range(dim)]
    for i in range(prob.n_comp):
        if (tid == i).any():
            continue
        nodes = np.flatnonzero(ftid == i)
        if nodes.size == 0:
            continue
        j = int(nodes[0])
        jk, stride, rem = 0, 1, j
        for d in range(dim):
            jd = rem % n[d]
            rem //= n[d]
            c, r = int(cmap[d][0][jd]), int(cmap[d][1][jd])
            kd = min(c + (1 if 2 * r >= n[d] - 1 else 0), nK[d] - 1)
            jk += kd * stride
            stride *= nK[d]
        if tid[jk] < 0:
            tid[jk] = i
            if g is not None:
                g = g.copy()
                g[jk] = np.asarray(prob.g)[j]
    def q1_axes(a):
        """A field with one value per node and axis, sampled axis by axis."""
        a = np.asarray(a).reshape(-1, dim)
        return np.stack([sample_q1(a[:, d], n, nK) for d in range(dim)], axis=1)

    drift = None if prob.drift is None else q1_axes(prob.drift)
    speed = prob.speed
    if speed is not None:
        speed = q1_axes(speed) if np.asarray(speed).ndim == 2 else q1(speed)
    ratio = max((n[d] - 1) / (nK[d] - 1) for d in range(dim))
    return prob.with_(name=prob.name + "_K", n=nK, target=tid, speed=speed,
                      cost=q1(prob.cost), g=g, drift=drift, h=prob.step * ratio,
                      coarse_stride=1, coarse_n=None)


def ra_delta(probK) -> float:
    """RA threshold 2 (C dx^q + M dx) of Proposition 3.1 on grid ``probK``."""
    dx = max(probK.dx)
    return 2.0 * (probK.ra_C * math.pow(dx, probK.ra_q) + probK.ra_M * dx)


def reconstruct_on(probK, delta: Optional[float] = None, tol: Optional[float] = None,
                   max_sweeps: int = 10**7):
    """RA steps 1-3 on the grid of ``probK``: auxiliary solves (to ``tol``, default
    the problem's ``ra_tol``), min, threshold.
    Returns (member bitmask, label, V_aux list, V, delta, sweeps)."""
    if delta is None:
        delta = ra_delta(probK)
    if tol is None:
        tol = probK.ra_tol
    fixed = fixed_mask(probK)
    V_aux, sweeps = [], []
    for i in range(probK.n_comp):                          # step 1
        Vi, _, s, _ = solve(probK, V0=initial_values(probK, comp=i), fixed=fixed, tol=tol,
                            max_sweeps=max_sweeps)
        V_aux.append(Vi)
        sweeps.append(s)
    V = V_aux[0].copy()                                    # step 2
    for Vi in V_aux[1:]:
        V = np.minimum(V, Vi)
    tid = np.asarray(probK.target)
    member = np.zeros(probK.N, dtype=np.uint8)             # step 3
    label = np.full(probK.N, 255, dtype=np.uint8)
    for i, Vi in enumerate(V_aux):
        sel = (tid == i) | (np.abs(Vi - V) <= delta)
        member |= (sel.astype(np.uint8) << i)
    for i in reversed(range(probK.n_comp)):                # lowest index wins ties
        label[V_aux[i] == V] = i
    return member, label, V_aux, V, delta, sweeps


def project(member_K: np.ndarray, label_K: np.ndarray, nK: tuple, n: tuple):
    """ISA step 2: Con(.) projection of the coarse sets to the fine grid (integer
    only), orphan repair, and the nearest-coarse-node label."""
    dim = len(n)
    mK = member_K.reshape(tuple(reversed(nK)))
    lK = label_K.reshape(tuple(reversed(nK)))
    # per coarse cell: AND and OR of the member bits of its 2^d corners
    cells_and = None
    cells_or = None
    for corner in range(1 << dim):
        sl = []
        for d in reversed(range(dim)):                     # numpy axis order
            b = (corner >> d) & 1
            sl.append(slice(b, nK[d] - 1 + b))
        v = mK[tuple(sl)]
        cells_and = v.copy() if cells_and is None else (cells_and & v)
        cells_or = v.copy() if cells_or is None else (cells_or | v)
    # per fine index and axis: the (up to two) coarse cells whose closure holds it
    cand, near = [], []
    for d in range(dim):
        c, r = coarse_coordinate_of_fine(n[d], nK[d])
        hi_c = np.minimum(c, nK[d] - 2)
        lo_c = np.where(r == 0, np.maximum(c - 1, 0), hi_c)
        cand.append((lo_c, hi_c))
        near.append(np.minimum(c + (2 * r >= n[d] - 1), nK[d] - 1))
    mem = np.zeros(tuple(reversed(n)), dtype=np.uint8)
    orf = np.zeros_like(mem)
    for choice in range(1 << dim):
        idx = [cand[d][(choice >> d) & 1] for d in range(dim)]
        ix = np.ix_(*reversed(idx))
        mem |= cells_and[ix]
        orf |= cells_or[ix]
    mem = np.where(mem == 0, orf, mem).astype(np.uint8)
    lab = lK[np.ix_(*reversed(near))]
    return mem.reshape(-1), np.ascontiguousarray(lab).reshape(-1)


def reconstruct(prob, delta: Optional[float] = None, max_sweeps: int = 10**7) -> Reconstruction:
    """ISA steps 1-2: RA on the coarse grid K, projection to the fine grid."""
    probK = coarse_problem(prob)
    mK, lK, V_aux, VK, delta, sweeps = reconstruct_on(probK, delta, max_sweeps=max_sweeps)
    mem, lab = project(mK, lK, probK.n, prob.n)
    return Reconstruction(mK, lK, V_aux, VK, delta, probK.n, mem, lab, sweeps)


def solve_subdomains(prob, member: np.ndarray, tol: float = 0.0, max_sweeps: int = 10**7,
                     want_policy: bool = False):
    """ISA step 3: V_i = T(V_i) on each projected set (non-members are ghosts)."""
    fixed = fixed_mask(prob)
    out, pols, sweeps = [], [], []
    for i in range(prob.n_comp):
        dom = ((member >> i) & 1).astype(np.uint8)
        Vi, pol, s, _ = solve(prob, V0=initial_values(prob), fixed=fixed, dom=dom, tol=tol,
                              max_sweeps=max_sweeps)
        out.append(Vi)
        pols.append(pol)
        sweeps.append(s)
    return (out, pols, sweeps) if want_policy else (out, sweeps)


def assemble(V_sub: List[np.ndarray], member: np.ndarray, G: float):
    """ISA step 4: Vbar(j) = min over the sets containing j; owner = lowest argmin."""
    N = member.size
    Vbar = np.full(N, np.inf)
    owner = np.full(N, 255, dtype=np.uint8)
    for i, Vi in enumerate(V_sub):
        on = ((member >> i) & 1).astype(bool)
        better = on & (Vi < Vbar)
        Vbar[better] = Vi[better]
        owner[better] = i
    Vbar[np.isinf(Vbar)] = G
    return Vbar, owner


def isa(prob, delta: Optional[float] = None, max_sweeps: int = 10**7):
    """The whole ISA: returns (Vbar, owner, Reconstruction, V_sub, sweeps)."""
    rec = reconstruct(prob, delta, max_sweeps=max_sweeps)
    V_sub, sweeps = solve_subdomains(prob, rec.member, max_sweeps=max_sweeps)
    Vbar, owner = assemble(V_sub, rec.member, prob.v_ghost)
    return Vbar, owner, rec, V_sub, sweeps


def adjoint_isa(prob, member: np.ndarray, pols: List[np.ndarray], owner: np.ndarray,
                gV: np.ndarray, tol: float = 0.0, max_iters: int = 10**7):
    """Gradient of a loss on the assembled value Vbar with respect to the running
    cost l, with the sets (``member``) and every set's policy frozen.  Vbar(j) is
    the owner set's value, so dL/dVbar is routed to the owner; each set then runs
    its own adjoint (non-members are ghosts, i.e. constants), and the per-set
    dL/dl add up.  Returns (dLdl, per-set adjoint states)."""
    from . import adjoint
    fixed = fixed_mask(prob)
    total = np.zeros(prob.N)
    lams = []
    for i in range(prob.n_comp):
        dom = ((member >> i) & 1).astype(np.uint8)
        gi = np.where(owner == i, gV, 0.0)
        lam_i, dLdl_i, _, _ = adjoint(prob, pols[i], gi, fixed=fixed, dom=dom, tol=tol,
                                      max_iters=max_iters)
        total += dLdl_i
        lams.append(lam_i)
    return total, lams


def split_component(target: np.ndarray, n: tuple, comp: int, new_label: int) -> np.ndarray:
    """Halve target component ``comp``: along the grid axis on which its nodes span
    the most index positions (lowest axis on ties), order the nodes by (index on
    that axis, flat index) and give the upper floor(count/2) of them ``new_label``."""
    dim = len(n)
    tid = np.asarray(target).copy()
    nodes = np.flatnonzero(tid == comp)
    idx = []
    rem = nodes.copy()
    for d in range(dim):
        idx.append(rem % n[d])
        rem //= n[d]
    extent = [int(idx[d].max() - idx[d].min()) for d in range(dim)]
    axis = int(np.argmax(extent))                     # first maximum: lowest axis
    order = np.lexsort((nodes, idx[axis]))            # by axis index, then flat index
    upper = nodes[order[len(nodes) - len(nodes) // 2:]]
    tid[upper] = new_label
    return tid


def refine_split(prob, max_comp: int, frac_goal: float = 0.0):
    """Recursive refinement of the division of Gamma for balance (the remedy the
    paper's conclusions propose for unbalanced sets): after each reconstruction,
    the component whose projected set holds the most fine nodes (lowest index on
    ties) among those with at least two target nodes is halved
    (``split_component``), until there are ``max_comp`` components or the largest
    set fraction is at most ``frac_goal``.

    Returns (target ids, component count, largest set fraction after each
    reconstruction)."""
    tid = np.asarray(prob.target).astype(np.int8).copy()
    nc = int(prob.n_comp)
    history = []
    while True:
        rec = reconstruct(prob.with_(target=tid, n_comp=nc))
        counts = np.array([int(((rec.member >> i) & 1).sum()) for i in range(nc)])
        history.append(float(counts.max()) / prob.N)
        if nc >= max_comp or history[-1] <= frac_goal:
            break
        sizes = np.array([int((tid == i).sum()) for i in range(nc)])
        cands = [i for i in sorted(range(nc), key=lambda i: (-counts[i], i)) if sizes[i] >= 2]
        if not cands:
            break
        tid = split_component(tid, tuple(prob.n[:prob.dim]), cands[0], nc)
        nc += 1
    return tid, nc, history
