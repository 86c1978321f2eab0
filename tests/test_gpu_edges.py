"""Edge cases of the GPU path against the oracle: an empty target component, the
largest control table (256 controls), the largest game table (64 x 64 rows) and
an evader with a single choice."""
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


def host(t):
    return t.detach().cpu().numpy()


def ra_of(p):
    return S.RaOpts(coarse_stride=p.coarse_stride, coarse_n=p.coarse_n, C=p.ra_C, M=p.ra_M,
                    q=p.ra_q, tol=p.ra_tol)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_empty_component(dtype):
    """Component 1 of 4 has no target node: its set is empty and no label names it;
    everything else matches the oracle (FP64 bit-exact, FP32 within 1e-5)."""
    p = W.c2_multitarget(n=65, m=16)
    tid = np.asarray(p.target).copy()
    tid[tid == 1] = -1
    p = p.with_(target=tid)
    say("case: empty component", dtype)
    V, owner, member, label, _, _, st = S.isa(S.to_device(p, dtype), ra_of(p),
                                              S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vbar, own_o, rec, _, _ = I.isa(p)
    assert st["converged"]
    assert np.array_equal(host(member), rec.member)
    assert np.array_equal(host(label), rec.label)
    assert not ((host(member) >> 1) & 1).any()
    if dtype == torch.float64:
        assert np.array_equal(host(V), Vbar)
    else:
        assert np.abs(host(V).astype(np.float64) - Vbar).max() <= 1e-5


def test_largest_control_table():
    """m = 256 (SL_MAX_CONTROLS) unit directions, FP64 global solve bit-exact."""
    p = W.c2_multitarget(n=33, m=256)
    say("case: 256 controls")
    V, _, st = S.solve(S.to_device(p, torch.float64), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, _, _ = O.solve(p)
    assert st["converged"]
    assert np.array_equal(host(V), Vo)


def test_largest_game_table():
    """64 pursuer controls x 64 evader choices = 4096 rows (SL_MAX_TABLE): FP64
    bit-exact and FP32 within 1e-5."""
    X = W.node_coords((33, 33), (-1.0, -1.0), (1.0, 1.0))
    p = W.pursuit_evasion_problem(33, split=1, m_a=64, m_b=63).with_(
        speed=W.f32(1.0 + 0.2 * X[:, 0] ** 2))
    assert p.m * np.asarray(p.velocity_b).shape[0] == 4096
    say("case: 4096-row game")
    Vo, _, _, _ = O.solve(p)
    V64, _, st = S.solve(S.to_device(p, torch.float64), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    assert st["converged"] and np.array_equal(host(V64), Vo)
    V32, _, st = S.solve(S.to_device(p, torch.float32), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    assert st["converged"] and np.abs(host(V32).astype(np.float64) - Vo).max() <= 1e-5


def test_single_choice_evader_is_a_drifted_control_problem():
    """An evader with one choice b0: f = c (a - b0), i.e. the control problem with
    the constant drift -c b0 folded into the table; FP64 bit-exact against the
    oracle's game operator."""
    p = W.c2_multitarget(n=65, m=16).with_(velocity_b=np.array([[0.25, -0.1]]))
    V, _, st = S.solve(S.to_device(p, torch.float64), S.SolveOpts(tol=0.0, max_sweeps=CAP))
    Vo, _, _, _ = O.solve(p)
    assert st["converged"]
    assert np.array_equal(host(V), Vo)
