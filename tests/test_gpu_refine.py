"""Recursive refinement of the target split (sl_refine_split) on the GPU against
the oracle: refined target ids, component count and the largest set fraction after
every reconstruction, bit for bit."""
import numpy as np
import pytest
import torch

import paper_1405_3521_amd as S
import workloads as W
from oracle import isa as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def ra_of(p):
    return S.RaOpts(coarse_stride=p.coarse_stride, coarse_n=p.coarse_n, C=p.ra_C, M=p.ra_M,
                    q=p.ra_q, tol=p.ra_tol)


@pytest.mark.parametrize("case", ["vdp129", "box65", "aniso3d17", "vdp97_goal"])
def test_refine_split_matches_oracle(case):
    goal = 0.0
    if case == "vdp129":
        p, mc = W.vdp_problem(129, split=1).with_(coarse_stride=4, ra_C=0.05, ra_M=0.05), 8
    elif case == "box65":
        p, mc = W.box_distance_problem(65, split=1).with_(coarse_stride=4), 4
    elif case == "aniso3d17":
        p, mc = W.c3_aniso3d(n=17, m=32, n_balls=2, r=0.2).with_(coarse_stride=4), 5
    else:
        p, mc, goal = W.vdp_problem(97, split=2).with_(coarse_n=(25, 25), ra_C=0.05,
                                                        ra_M=0.05), 8, 0.55
    say("case: refine", case)
    tid_o, nc_o, hist_o = I.refine_split(p, mc, frac_goal=goal)
    dp = S.to_device(p, torch.float32)
    tid, nc, hist, st = S.refine_split(dp, ra_of(p), mc, frac_goal=goal)
    say("  components", nc, "largest set fractions", [round(h, 3) for h in hist])
    assert nc == nc_o
    assert np.array_equal(tid.cpu().numpy(), tid_o)
    assert hist == hist_o
