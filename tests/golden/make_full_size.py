"""Writes the expected values of the full-size GPU parity tests, from the FP64
oracle alone.

    python tests/golden/make_full_size.py [NAME ...]     # default: every case

Each case writes ``<NAME>.npz`` next to this script.  Nothing here touches the HIP
library: the inputs come from ``workloads`` (seeded data) and every stored number
from ``oracle`` (the plain FP64 implementation of the scheme, the reconstruction
algorithm of Sec. 3 and the independent-sets algorithm of Sec. 4).  The solves
run to stagnation (a sweep that changes nothing), as the parity bar asks.

Storage: values are the oracle's FP64 results rounded to the nearest float32
(an absolute change of at most 2^-25 for values below 1 and 2^-24 below 2),
which the 1e-5 value bar absorbs; integer outputs (sets, labels, owners) are
stored exactly.  Per-set values are kept where they matter beyond the assembly:
on member nodes whose owner is another set.

Cases
  c2_1025     the headline problem (1025^2, 64 controls, 4 disks): ISA to
              stagnation, V-bar, owner, sets, labels, per-set values
  c2_513      the same workload at 513^2
  c3_257_ra   the 3D workload (257^3): the coarse reconstruction on 65^3
              (sets and labels on K; the fine sets follow by the Con projection)
  c4_large    a sub-batch of the 512-problem batch: its three largest problems
              (sides >= 400) and five smaller ones, ISA each
  c5_513      the gradient workload at 513^2 (ISA forward, sets frozen): the
              loss's gradient with respect to theta by the FP64 adjoint, and
              central differences along 8 dense directions (eps = 1e-4 and
              1e-6) and 8 single nodes (eps = 1e-4), each with the number of
              argmin switches inside +-eps
  c5_129      the same at 129^2 with 8 directions and 32 single nodes
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O          # noqa: E402
import workloads as W       # noqa: E402
from oracle import isa as I  # noqa: E402

FD_EPS = 1e-4
# a second, smaller step along the dense directions: at 1e-4 a dense direction
# moves the near-tied candidates of some nodes past each other, so L has a kink
# inside +-eps there; the switch count of every difference is stored with it
FD_EPS_SMALL = 1e-6
FD_SEED = 705


def say(*a):
    print(*a, flush=True)


def _isa_arrays(p):
    """The oracle's ISA of problem p as the arrays a parity test compares."""
    t0 = time.time()
    Vbar, owner, rec, Vs, sweeps = I.isa(p)
    idx, sets, vals = [], [], []
    for i, Vi in enumerate(Vs):
        on = ((rec.member >> i) & 1).astype(bool) & (owner != i)
        j = np.flatnonzero(on)
        idx.append(j.astype(np.int32))
        sets.append(np.full(j.size, i, dtype=np.uint8))
        vals.append(Vi[j].astype(np.float32))
    say(f"  {p.name}: ISA in {time.time() - t0:.0f} s, sweeps {sweeps}")
    return dict(V=Vbar.astype(np.float32), owner=owner, member=rec.member, label=rec.label,
                member_K=rec.member_K, label_K=rec.label_K,
                other_idx=np.concatenate(idx), other_set=np.concatenate(sets),
                other_val=np.concatenate(vals), sweeps=np.asarray(sweeps, dtype=np.int64),
                n=np.asarray(p.n, dtype=np.int64))


def case_c2_1025():
    return _isa_arrays(W.c2_multitarget())


def case_c2_513():
    return _isa_arrays(W.c2_multitarget(n=513, m=64))


def case_c3_257_ra():
    p = W.c3_aniso3d()
    t0 = time.time()
    probK = I.coarse_problem(p)
    mK, lK, _, _, delta, sweeps = I.reconstruct_on(probK)
    say(f"  c3 RA on {probK.n} in {time.time() - t0:.0f} s, sweeps {sweeps}")
    return dict(member_K=mK, label_K=lK, nK=np.asarray(probK.n, dtype=np.int64),
                delta=np.float64(delta), sweeps=np.asarray(sweeps, dtype=np.int64))


# the three largest problems of the batch and five smaller ones spread over the
# size range (the smallest included)
def c4_subset():
    probs = W.c4_batch()
    sides = np.array([q.n[0] for q in probs])
    order = np.argsort(-sides, kind="stable")
    big = [int(k) for k in order[:3]]
    rest = order[3:]
    pick = [int(rest[k]) for k in np.linspace(0, rest.size - 1, 5).round().astype(int)]
    return big + pick, probs


def case_c4_large():
    ids, probs = c4_subset()
    out = {"ids": np.asarray(ids, dtype=np.int64)}
    for k in ids:
        a = _isa_arrays(probs[k])
        for key in ("V", "owner", "member", "label"):
            out[f"p{k}_{key}"] = a[key]
    return out


def _c5_gradient(p, n_dirs: int, n_nodes: int):
    """ISA forward with the sets of the reconstruction frozen; loss
    sum (V-bar[obs] - V_obs)^2; gradient with respect to theta (l = e^theta) by the
    per-set adjoints; central differences of the loss."""
    rec = I.reconstruct(p)
    member = rec.member
    obs = p.meta["obs"]
    th = p.meta["theta"]

    def fwd(theta, want_policy=False):
        q = p.with_(cost=np.exp(theta))
        Vs, pols, _ = I.solve_subdomains(q, member, want_policy=True)
        Vbar, owner = I.assemble(Vs, member, q.v_ghost)
        return Vbar, owner, pols

    t0 = time.time()
    Vt, _, _ = fwd(p.meta["theta_true"])
    Vobs = Vt[obs]
    Vbar, owner, pols = fwd(th)
    say(f"  {p.name}: two forwards in {time.time() - t0:.0f} s")
    gV = np.zeros(p.N)
    gV[obs] = 2.0 * (Vbar[obs] - Vobs)
    dLdl, _ = I.adjoint_isa(p.with_(cost=np.exp(th)), member, pols, owner, gV)
    grad = dLdl * np.exp(th)

    def central(step):
        """Central difference of the loss along `step` (already scaled by eps), and
        the number of (set, node) pairs whose argmin control differs from the base
        policy in either of the two solves (a kink of L within +-eps)."""
        Vp, _, pp = fwd(th + step)
        Vm, _, pm = fwd(th - step)
        Lp = float(np.sum((Vp[obs] - Vobs) ** 2))
        Lm = float(np.sum((Vm[obs] - Vobs) ** 2))
        switched = sum(int(((a != b) | (c != b)).sum()) for a, b, c in zip(pp, pols, pm))
        return Lp - Lm, switched

    rng = np.random.Generator(np.random.PCG64(FD_SEED))
    dirs = rng.normal(size=(n_dirs, p.N))
    free = np.flatnonzero(np.asarray(p.target) < 0)
    nodes = np.sort(rng.choice(np.intersect1d(free, obs), size=n_nodes, replace=False))
    fd_dir = np.empty(n_dirs)
    fd_dir_small = np.empty(n_dirs)
    sw_dir = np.zeros(n_dirs, dtype=np.int64)
    sw_dir_small = np.zeros(n_dirs, dtype=np.int64)
    for k in range(n_dirs):
        dL, sw_dir[k] = central(FD_EPS * dirs[k])
        fd_dir[k] = dL / (2 * FD_EPS)
        dL, sw_dir_small[k] = central(FD_EPS_SMALL * dirs[k])
        fd_dir_small[k] = dL / (2 * FD_EPS_SMALL)
        say(f"    direction {k}: adjoint {grad @ dirs[k]:.9e} fd(1e-4) {fd_dir[k]:.9e} "
            f"[{sw_dir[k]} switched] fd(1e-6) {fd_dir_small[k]:.9e} [{sw_dir_small[k]}]")
    fd_node = np.empty(n_nodes)
    sw_node = np.zeros(n_nodes, dtype=np.int64)
    for k, j in enumerate(nodes):
        e = np.zeros(p.N)
        e[j] = FD_EPS
        dL, sw_node[k] = central(e)
        fd_node[k] = dL / (2 * FD_EPS)
        say(f"    node {j}: adjoint {grad[j]:.9e} fd {fd_node[k]:.9e} [{sw_node[k]} switched]")
    return dict(member=member, owner=owner, V=Vbar.astype(np.float32), V_obs=Vobs,
                grad=grad, loss=np.float64(np.sum((Vbar[obs] - Vobs) ** 2)),
                dir_seed=np.int64(FD_SEED), eps=np.float64(FD_EPS), fd_dir=fd_dir,
                switched_dir=sw_dir, eps_small=np.float64(FD_EPS_SMALL),
                fd_dir_small=fd_dir_small, switched_dir_small=sw_dir_small,
                nodes=nodes.astype(np.int64), fd_node=fd_node, switched_node=sw_node)


def case_c5_513():
    return _c5_gradient(W.c5_adjoint(), n_dirs=8, n_nodes=8)


def case_c5_129():
    return _c5_gradient(W.c5_adjoint(n=129, n_obs=1500), n_dirs=8, n_nodes=32)


CASES = {
    "c2_513": case_c2_513,
    "c5_129": case_c5_129,
    "c3_257_ra": case_c3_257_ra,
    "c4_large": case_c4_large,
    "c2_1025": case_c2_1025,
    "c5_513": case_c5_513,
}


def path_of(name: str) -> str:
    return os.path.join(HERE, f"{name}.npz")


def main(names):
    say(f"oracle threads: {O.max_threads()}")
    for name in names or list(CASES):
        t0 = time.time()
        say(f"case {name}")
        arrays = CASES[name]()
        np.savez_compressed(path_of(name), **arrays)
        say(f"case {name}: written in {time.time() - t0:.0f} s "
            f"({os.path.getsize(path_of(name)) / 1e6:.2f} MB)")


if __name__ == "__main__":
    main(sys.argv[1:])
