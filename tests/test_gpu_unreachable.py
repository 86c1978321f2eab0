"""The count of unreachable nodes (sl_stats.n_unreachable): free nodes whose value
stays at the ghost value up to rounding (8 eps v_ghost / (1 - beta)), because no
trajectory from them reaches a target.  A block of nodes with zero speed cannot move, so each of them
keeps the ghost value; the count equals the oracle's count of the same nodes, in
the global solve and in the ISA."""
import numpy as np
import pytest
import torch

import oracle as O
import paper_1405_3521_amd as S
import workloads as W
from oracle import isa as I

pytestmark = pytest.mark.gpu

CAP = 50_000


def say(*a):
    print(*a, flush=True)


def _problem():
    p = W.c2_multitarget(n=65, m=32)
    sp = p.speed.copy().reshape(65, 65)
    tgt = np.asarray(p.target).reshape(65, 65)
    blk = (slice(2, 7), slice(2, 7))          # a 5x5 corner block away from the disks
    assert (tgt[blk] < 0).all()
    sp[blk] = 0.0
    return p.with_(speed=sp.reshape(-1))


def _oracle_count(p, V, eps):
    free = np.asarray(p.target) < 0
    beta, _ = O.scheme_constants(p.lam, p.step, p.disc)
    return int((free & (V >= p.v_ghost - 8 * eps * abs(p.v_ghost) / (1 - beta))).sum())


@pytest.mark.parametrize("dtype,eps", [(torch.float32, 2.0 ** -23), (torch.float64, 2.0 ** -52)])
def test_unreachable_count(dtype, eps):
    p = _problem()
    say("case: unreachable count", dtype)
    Vo, _, _, _ = O.solve(p)
    n_o = _oracle_count(p, Vo, 2.0 ** -52)
    assert n_o == 25
    dp = S.to_device(p, dtype)
    V, _, st = S.solve(dp, S.SolveOpts(tol=0.0, max_sweeps=CAP))
    say("  global", st["n_unreachable"], "oracle", n_o)
    assert st["converged"] and st["n_unreachable"] == n_o
    ra = S.RaOpts(coarse_stride=p.coarse_stride, coarse_n=p.coarse_n, C=p.ra_C, M=p.ra_M,
                  q=p.ra_q, tol=p.ra_tol)
    Vb, owner, member, label, _, _, st = S.isa(dp, ra, S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vbo, _, _, _, _ = I.isa(p)
    n_io = _oracle_count(p, Vbo, 2.0 ** -52)
    say("  isa", st["n_unreachable"], "oracle", n_io)
    assert st["n_unreachable"] == n_io
