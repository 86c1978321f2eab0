"""Pins of the oracle's policy-frozen adjoint and tangent (no GPU).

With the argmin policy frozen, the fixed point is linear in the running cost l:
V = beta P V + w l + const on free nodes, so a loss L(V) has
dL/dl = w lambda with lambda = dL/dV + beta P^T lambda."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as O
import workloads as W
from oracle import isa as I


VARIANTS = {
    "plain": dict(),
    "swirl": dict(swirl=0.5),          # drift: feet shift by q_j per node
    "axes": dict(axis_speed=True),     # S(x) = diag(c_1, c_2)
}


@pytest.fixture(scope="module", params=list(VARIANTS))
def prob(request):
    return W.c5_adjoint(n=65, n_obs=300, **VARIANTS[request.param])


def _linear_system(p, pol, dom=None):
    """Sparse (I - beta P) on free nodes and the constant part of the right side."""
    beta, w = O.scheme_constants(p.lam, p.step, p.disc)
    cidx, wts = O.policy_stencil(p, pol, dom=dom)
    fixed = O.fixed_mask(p).astype(bool)
    free = (pol >= 0)
    pos = -np.ones(p.N, dtype=np.int64)
    pos[free] = np.arange(free.sum())
    V0 = O.initial_values(p)
    rows, cols, vals = [], [], []
    const = np.zeros(free.sum())
    fj = np.flatnonzero(free)
    for s in range(cidx.shape[1]):
        c = cidx[fj, s]
        wt = wts[fj, s]
        ghost = c < 0
        const += np.where(ghost, beta * wt * p.v_ghost, 0.0)
        cc = np.where(ghost, 0, c)
        fx = ~ghost & fixed[cc]
        const += np.where(fx, beta * wt * V0[cc], 0.0)
        fr = ~ghost & ~fixed[cc]
        rows.append(pos[fj[fr]])
        cols.append(pos[cc[fr]])
        vals.append(beta * wt[fr])
    nf = free.sum()
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(nf, nf))
    A = sp.identity(nf, format="csr") - P
    l = np.ones(p.N) if p.cost is None else p.cost
    return A, const + w * l[free], free, w


def test_forward_equals_policy_linear_solve(prob):
    """The policy stencil reproduces the fixed point: (I - beta P) V = w l + const."""
    V, pol, _, _ = O.solve(prob)
    A, rhs, free, _ = _linear_system(prob, pol)
    x = spla.spsolve(A.tocsc(), rhs)
    assert np.abs(x - V[free]).max() <= 1e-12


def test_adjoint_equals_sparse_lu(prob):
    """Jacobi adjoint = direct solve of (I - beta P)^T lambda = g."""
    V, pol, _, _ = O.solve(prob)
    rng = np.random.Generator(np.random.PCG64(3))
    gV = np.zeros(prob.N)
    obs = prob.meta["obs"]
    gV[obs] = rng.normal(size=obs.size)
    lam, dLdl, it, _ = O.adjoint(prob, pol, gV)
    A, _, free, w = _linear_system(prob, pol)
    x = spla.spsolve(A.T.tocsc(), gV[free])
    assert np.abs(lam[free] - x).max() <= 1e-12 * max(1.0, np.abs(x).max())
    assert np.abs(dLdl - w * lam).max() == 0.0
    assert (lam[~free] == 0).all()


def test_dot_product_tangent_adjoint(prob):
    """<lambda, w dl> = <g, Vdot> for the tangent Vdot = beta P Vdot + w dl."""
    V, pol, _, _ = O.solve(prob)
    rng = np.random.Generator(np.random.PCG64(4))
    gV = rng.normal(size=prob.N)
    dl = rng.normal(size=prob.N)
    lam, dLdl, _, _ = O.adjoint(prob, pol, gV)
    Vdot, _ = O.tangent(prob, pol, dl)
    lhs = float(np.dot(dLdl, dl))
    rhs = float(np.dot(gV, Vdot))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_adjoint_nonnegative(prob):
    """g >= 0 => lambda >= 0 (P and beta are non-negative)."""
    V, pol, _, _ = O.solve(prob)
    rng = np.random.Generator(np.random.PCG64(5))
    gV = rng.random(prob.N)
    lam, _, _, _ = O.adjoint(prob, pol, gV)
    assert lam.min() >= 0.0


def _loss(p, theta, obs, Vobs):
    V, pol, _, _ = O.solve(p.with_(cost=np.exp(theta)))
    return float(np.sum((V[obs] - Vobs) ** 2)), V, pol


def test_gradient_against_central_fd(prob):
    """dL/dtheta (adjoint, l = exp(theta)) against central finite differences of the
    FP64 forward solve: eps = 1e-4 along single-node directions, eps = 1e-6 along
    dense random directions (at 1e-4 a dense direction flips the argmin at ~10
    near-tied nodes, where L is only piecewise smooth).  Cases without a policy
    switch inside +-eps must agree to 1e-6 relative; switched cases are bounded
    loosely and counted."""
    p = prob
    th = p.meta["theta"]
    obs = p.meta["obs"]
    Vtrue, _, _, _ = O.solve(p.with_(cost=np.exp(p.meta["theta_true"])))
    Vobs = Vtrue[obs]
    L0, V, pol = _loss(p, th, obs, Vobs)
    gV = np.zeros(p.N)
    gV[obs] = 2.0 * (V[obs] - Vobs)
    _, dLdl, _, _ = O.adjoint(p.with_(cost=np.exp(th)), pol, gV)
    grad = dLdl * np.exp(th)
    rng = np.random.Generator(np.random.PCG64(705))
    cases = [(rng.normal(size=p.N), 1e-6) for _ in range(4)]
    free = np.flatnonzero(pol >= 0)
    near_obs = np.intersect1d(free, obs)
    for j in rng.choice(near_obs, size=6, replace=False):
        e = np.zeros(p.N)
        e[j] = 1.0
        cases.append((e, 1e-4))
    clean = 0
    for d, eps in cases:
        Lp, _, pp = _loss(p, th + eps * d, obs, Vobs)
        Lm, _, pm = _loss(p, th - eps * d, obs, Vobs)
        fd = (Lp - Lm) / (2 * eps)
        an = float(np.dot(grad, d))
        switched = (pp != pol).any() or (pm != pol).any()
        tol = 2e-2 if switched else 1e-6
        assert abs(fd - an) <= tol * max(abs(an), 1e-10), (fd, an, eps, switched)
        clean += not switched
    assert clean >= 0.75 * len(cases)


def test_isa_gradient_against_fd():
    """The same for the ISA forward (sets frozen): dL/dVbar routed to the owner
    set, per-set adjoints summed."""
    p = W.c5_adjoint(n=65, n_obs=300)
    rec = I.reconstruct(p)
    obs = p.meta["obs"]
    th = p.meta["theta"]

    def fwd(theta):
        q = p.with_(cost=np.exp(theta))
        Vs, pols, _ = I.solve_subdomains(q, rec.member, want_policy=True)
        Vbar, owner = I.assemble(Vs, rec.member, q.v_ghost)
        return Vbar, owner, pols

    Vt, _, _ = fwd(p.meta["theta_true"])
    Vobs = Vt[obs]
    Vbar, owner, pols = fwd(th)
    gV = np.zeros(p.N)
    gV[obs] = 2.0 * (Vbar[obs] - Vobs)
    dLdl, _ = I.adjoint_isa(p.with_(cost=np.exp(th)), rec.member, pols, owner, gV)
    grad = dLdl * np.exp(th)
    rng = np.random.Generator(np.random.PCG64(706))
    eps = 1e-6
    for _ in range(3):
        d = rng.normal(size=p.N)
        Vp, op, _ = fwd(th + eps * d)
        Vm, om, _ = fwd(th - eps * d)
        fd = (np.sum((Vp[obs] - Vobs) ** 2) - np.sum((Vm[obs] - Vobs) ** 2)) / (2 * eps)
        an = float(np.dot(grad, d))
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


@pytest.mark.parametrize("case", ["c5_129", "c5_513"])
def test_stored_gradient_against_stored_differences(case):
    """The oracle's ISA gradient of the learnable-cost workload against the oracle's
    own central differences, both stored by tests/golden/make_full_size.py
    (eps = 1e-4 along single nodes (32 at 129^2, 8 at 513^2) and 8 dense
    directions, eps = 1e-6 along the same directions).  Where no argmin switches inside +-eps the two agree to
    1e-6 relative; a dense direction at eps = 1e-4 moves the near-tied candidates
    of tens of nodes past each other (L has kinks there), so it is only counted,
    and at eps = 1e-6 (one or two switches) it agrees to 1e-2."""
    import os
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", f"{case}.npz"))
    grad = g["grad"]
    n_single = 0
    for j, fd, sw in zip(g["nodes"], g["fd_node"], g["switched_node"]):
        if sw == 0:
            assert abs(fd - grad[j]) <= 1e-6 * abs(grad[j]), (j, fd, grad[j])
            n_single += 1
    assert n_single >= 0.75 * len(g["nodes"])
    N = grad.size
    rng = np.random.Generator(np.random.PCG64(int(g["dir_seed"])))
    dirs = rng.normal(size=(len(g["fd_dir"]), N))
    for k, d in enumerate(dirs):
        an = float(grad @ d)
        if g["switched_dir"][k] == 0:
            assert abs(g["fd_dir"][k] - an) <= 1e-6 * abs(an)
        if g["switched_dir_small"][k] == 0:
            assert abs(g["fd_dir_small"][k] - an) <= 1e-6 * abs(an)
        else:
            assert abs(g["fd_dir_small"][k] - an) <= 1e-2 * abs(an)
