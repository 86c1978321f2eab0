"""Writes the fine reference of the Van der Pol accuracy table (Sec. 4.1, Tab. 5),
from the FP64 oracle alone.

    python tests/golden/make_vdp_reference.py      # writes vdp_401.npz here

The paper measures the error of the scheme on 50^2, 100^2 and 200^2 grids
against a 400^2 solution.  Here the reference is the oracle's global solve of the
same problem (Van der Pol dynamics with a control on the second component,
l = |x|, capture disk of radius 0.2, 21 controls, h = dx) on 401^2 nodes of
[-1, 1]^2, iterated until nothing changes.  The grids 51^2, 101^2 and 201^2 are
nested in it (every 8th, 4th and 2nd node), so errors are taken at coincident
nodes.  Values are stored as float32 (the table's errors are of order 1e-2).
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

N_REF = 401


def main():
    p = W.vdp_problem(N_REF, split=1)
    t0 = time.time()
    V, _, sweeps, res = O.solve(p)
    print(f"vdp {N_REF}^2: {sweeps} sweeps, residual {res}, {time.time() - t0:.0f} s", flush=True)
    path = os.path.join(HERE, f"vdp_{N_REF}.npz")
    np.savez_compressed(path, V=V.astype(np.float32), n=np.int64(N_REF),
                        v_ghost=np.float64(p.v_ghost), sweeps=np.int64(sweeps))
    print(path, os.path.getsize(path), flush=True)


if __name__ == "__main__":
    main()
