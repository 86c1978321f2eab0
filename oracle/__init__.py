"""FP64 CPU oracle for the semi-Lagrangian HJB solver and its sub-domain method.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product (``paper_1405_3521_amd``)
never does, and this package never imports the product.  It shares no code with
the HIP library; the only common module is ``workloads`` (seeded problem data,
no scheme arithmetic).

Layout
------
* ``sl_oracle.c``  -- the SL operator T (paper Sec. 3, (SL)/(Tdef)), its Jacobi
  iteration, the policy-frozen adjoint and tangent; built with gcc by ``build.py``.
* this module      -- ctypes bindings plus the node sets of each solve mode.
* ``isa.py``       -- the reconstruction algorithm (RA, Sec. 3) and the
  independent-sets algorithm (ISA, Sec. 4) as the paper lists their steps.
* ``tiny.py``      -- exact rational policy iteration for tiny grids (a pin).

Parity status: every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` (closed forms, brute force, invariants); none is
"parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Tuple

import numpy as np

from . import build as _build

_LIB = None
_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int)
_U8P = C.POINTER(C.c_uint8)
_I32P = C.POINTER(C.c_int32)
_I64P = C.POINTER(C.c_int64)

DISC = {"exp": 0, "paper": 1, "kruzkov": 2}
INTERP = {"q1": 0, "p1": 1}


def lib():
    """Load (building with gcc if absent) the oracle shared library."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.orc_scheme_constants.argtypes = [C.c_double, C.c_double, C.c_int, _DP, _DP]
        L.orc_scheme_constants.restype = C.c_int
        L.orc_max_threads.restype = C.c_int
        common = [C.c_int, _IP, _DP, _DP, C.c_double, C.c_int, _DP, _DP, C.c_int, _DP, C.c_int,
                  C.c_int]
        L.orc_apply.argtypes = common + [_DP, _DP, C.c_double, C.c_int, C.c_double, _U8P, _U8P,
                                         _DP, _DP, _I32P, C.c_int]
        L.orc_apply.restype = C.c_int
        L.orc_solve.argtypes = common + [_DP, _DP, C.c_double, C.c_int, C.c_double, _U8P, _U8P,
                                         _DP, _I32P, C.c_double, C.c_long, _DP, C.c_int]
        L.orc_solve.restype = C.c_long
        L.orc_policy_stencil.argtypes = common + [_DP, _U8P, _I32P, _I64P, _DP]
        L.orc_policy_stencil.restype = C.c_int
        L.orc_adjoint.argtypes = common + [_DP, C.c_double, C.c_int, _U8P, _U8P, _I32P, _DP,
                                           _DP, _DP, C.c_double, C.c_long, _DP]
        L.orc_adjoint.restype = C.c_long
        L.orc_tangent.argtypes = common + [_DP, C.c_double, C.c_int, _U8P, _U8P, _I32P, _DP,
                                           _DP, C.c_double, C.c_long, _DP]
        L.orc_tangent.restype = C.c_long
        _LIB = L
    return _LIB


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def _geom(prob):
    n = np.zeros(3, dtype=np.int32)
    lo = np.zeros(3)
    hi = np.ones(3)
    n[:prob.dim] = prob.n
    lo[:prob.dim] = prob.lo
    hi[:prob.dim] = prob.hi
    return n, lo, hi


def _common(prob):
    """Geometry, the pursuer's table, the speed (per node, or per node and axis) and
    the evader's table (none for a control problem)."""
    n, lo, hi = _geom(prob)
    b = np.ascontiguousarray(prob.velocity, dtype=np.float64)
    c = _f64(prob.speed)
    c_axes = 0
    if c is not None and c.ndim == 2:
        if c.shape != (prob.N, prob.dim):
            raise ValueError("per-axis speed must have shape (N, dim)")
        c_axes = 1
        c = np.ascontiguousarray(c.reshape(-1))
    vb = getattr(prob, "velocity_b", None)
    bb = None if vb is None else np.ascontiguousarray(vb, dtype=np.float64)
    mb = 0 if bb is None else int(bb.shape[0])
    keep = (n, lo, hi, b, c, bb)
    return keep, [prob.dim, _p(n, _IP), _p(lo, _DP), _p(hi, _DP), float(prob.step), prob.m,
                  _p(b, _DP), _p(c, _DP), mb, _p(bb, _DP), c_axes,
                  INTERP[getattr(prob, "interp", "q1")]]


def max_threads() -> int:
    return int(lib().orc_max_threads())


def scheme_constants(lam: float, h: float, disc: str = "exp") -> Tuple[float, float]:
    """(beta, w): discount and running-cost weight of one SL step of length h."""
    b = C.c_double()
    w = C.c_double()
    rc = lib().orc_scheme_constants(lam, h, DISC[disc], C.byref(b), C.byref(w))
    if rc:
        raise ValueError("invalid lam/h/disc")
    return b.value, w.value


# ------------------------------------------------------------------ solve modes
def fixed_mask(prob) -> np.ndarray:
    """Target nodes (of any component) keep their value in every mode."""
    return (np.asarray(prob.target) >= 0).astype(np.uint8)


def initial_values(prob, comp: Optional[int] = None) -> np.ndarray:
    """V^0: ghost value on free nodes, g on target nodes.  With ``comp`` given (an
    auxiliary problem of the RA), only that component's nodes hold g and the other
    components' nodes hold the ghost value (g_i > g off Gamma_i, (gcond))."""
    G = float(prob.v_ghost)
    V = np.full(prob.N, G)
    tgt = np.asarray(prob.target)
    gv = np.zeros(prob.N) if prob.g is None else np.asarray(prob.g, dtype=np.float64)
    on = tgt >= 0 if comp is None else tgt == comp
    V[on] = gv[on]
    return V


def apply_T(prob, V, fixed=None, dom=None, nthreads: int = 0):
    """One application of T: returns (T(V), policy).  For a game the policy of a
    node is l m + k (evader choice l, pursuer control k)."""
    L = lib()
    keep, com = _common(prob)
    V = _f64(V)
    TV = np.empty(prob.N)
    pol = np.empty(prob.N, dtype=np.int32)
    l = _f64(prob.cost)
    dr = None if prob.drift is None else _f64(prob.drift).reshape(-1)
    fixed = fixed_mask(prob) if fixed is None else _u8(fixed)
    dom = _u8(dom)
    rc = L.orc_apply(*com, _p(l, _DP), _p(dr, _DP), float(prob.lam), DISC[prob.disc],
                     float(prob.v_ghost), _p(fixed, _U8P), _p(dom, _U8P), _p(V, _DP),
                     _p(TV, _DP), _p(pol, _I32P), nthreads)
    if rc:
        raise RuntimeError(f"orc_apply failed ({rc})")
    return TV, pol


def solve(prob, V0=None, fixed=None, dom=None, tol: float = 0.0, max_sweeps: int = 10**7,
          nthreads: int = 0):
    """Jacobi iteration of T to ``tol`` (0: until nothing changes).

    Returns (V, policy, sweeps, residual).  Default V0 and fixed set: the global
    problem (every target component fixed at g)."""
    L = lib()
    keep, com = _common(prob)
    V = initial_values(prob) if V0 is None else np.array(V0, dtype=np.float64, copy=True)
    pol = np.empty(prob.N, dtype=np.int32)
    l = _f64(prob.cost)
    dr = None if prob.drift is None else _f64(prob.drift).reshape(-1)
    fixed = fixed_mask(prob) if fixed is None else _u8(fixed)
    dom = _u8(dom)
    res = C.c_double()
    s = L.orc_solve(*com, _p(l, _DP), _p(dr, _DP), float(prob.lam), DISC[prob.disc],
                    float(prob.v_ghost), _p(fixed, _U8P), _p(dom, _U8P), _p(V, _DP),
                    _p(pol, _I32P), float(tol), int(max_sweeps), C.byref(res), nthreads)
    if s < 0:
        raise RuntimeError(f"orc_solve failed ({s})")
    return V, pol, int(s), res.value


def policy_stencil(prob, policy, dom=None):
    """Corner indices (-1 ghost) and Q1 weights at the foot of each node's control."""
    L = lib()
    keep, com = _common(prob)
    K = 1 << prob.dim
    cidx = np.empty((prob.N, K), dtype=np.int64)
    wts = np.empty((prob.N, K))
    pol = np.ascontiguousarray(policy, dtype=np.int32)
    dr = None if prob.drift is None else _f64(prob.drift).reshape(-1)
    dom = _u8(dom)
    rc = L.orc_policy_stencil(*com, _p(dr, _DP), _p(dom, _U8P), _p(pol, _I32P),
                              _p(cidx, _I64P), _p(wts, _DP))
    if rc:
        raise RuntimeError(f"orc_policy_stencil failed ({rc})")
    return cidx, wts


def adjoint(prob, policy, gV, fixed=None, dom=None, tol: float = 0.0,
            max_iters: int = 10**7):
    """Adjoint state lambda = gV + beta P^T lambda of the policy-frozen scheme and
    dL/dl = w lambda.  Returns (lambda, dLdl, iterations, residual)."""
    L = lib()
    keep, com = _common(prob)
    pol = np.ascontiguousarray(policy, dtype=np.int32)
    gV = _f64(gV)
    lam_out = np.empty(prob.N)
    dLdl = np.empty(prob.N)
    dr = None if prob.drift is None else _f64(prob.drift).reshape(-1)
    fixed = fixed_mask(prob) if fixed is None else _u8(fixed)
    dom = _u8(dom)
    res = C.c_double()
    it = L.orc_adjoint(*com, _p(dr, _DP), float(prob.lam), DISC[prob.disc], _p(fixed, _U8P),
                       _p(dom, _U8P), _p(pol, _I32P), _p(gV, _DP), _p(lam_out, _DP),
                       _p(dLdl, _DP), float(tol), int(max_iters), C.byref(res))
    if it < 0:
        raise RuntimeError(f"orc_adjoint failed ({it})")
    return lam_out, dLdl, int(it), res.value


def tangent(prob, policy, dl, fixed=None, dom=None, tol: float = 0.0, max_iters: int = 10**7):
    """Vdot = beta P Vdot + w dl on free nodes (policy frozen).  Returns (Vdot, iters)."""
    L = lib()
    keep, com = _common(prob)
    pol = np.ascontiguousarray(policy, dtype=np.int32)
    dl = _f64(dl)
    out = np.empty(prob.N)
    dr = None if prob.drift is None else _f64(prob.drift).reshape(-1)
    fixed = fixed_mask(prob) if fixed is None else _u8(fixed)
    dom = _u8(dom)
    res = C.c_double()
    it = L.orc_tangent(*com, _p(dr, _DP), float(prob.lam), DISC[prob.disc], _p(fixed, _U8P),
                       _p(dom, _U8P), _p(pol, _I32P), _p(dl, _DP), _p(out, _DP), float(tol),
                       int(max_iters), C.byref(res))
    if it < 0:
        raise RuntimeError(f"orc_tangent failed ({it})")
    return out, int(it)
