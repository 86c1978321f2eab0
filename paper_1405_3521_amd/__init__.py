"""MI355X semi-Lagrangian HJB solver with independent sub-domains.

Thin Python binding of the C-ABI library ``libslhjb.so`` (declared in
``include/slhjb.h``).  PyTorch provides device memory and streams; every step of
the solver runs in the library's HIP kernels.  This module only marshals
arguments (ctypes) and allocates the output tensors and workspaces.

If the library is not built, or no HIP device is present, the functions raise:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

__all__ = [
    "DeviceProblem", "RaOpts", "SolveOpts", "lib", "lib_path", "to_device", "solve",
    "solve_noalloc",
    "reconstruct", "solve_isa", "isa", "adjoint", "solve_batched", "BatchedSolver",
    "refine_split", "SlError",
    "HJBSolve",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_lib", "libslhjb.so")
_LIB = None

SL_OK, SL_NOT_CONVERGED = 0, 1
DISC = {"exp": 0, "paper": 1, "kruzkov": 2}
INTERP = {"q1": 0, "p1": 1}
ABI_VERSION = 5          # struct layout of slhjb.h


class SlError(RuntimeError):
    def __init__(self, fn: str, status: int):
        msg = lib().sl_status_string(status).decode()
        super().__init__(f"{fn} failed: {msg} ({status})")
        self.status = status


class SlProblem(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("n", C.c_int * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("m", C.c_int), ("velocity", C.POINTER(C.c_double)), ("speed", C.c_void_p),
        ("cost", C.c_void_p), ("drift", C.c_void_p), ("target", C.c_void_p), ("g", C.c_void_p),
        ("n_comp", C.c_int), ("lambda_", C.c_double), ("h", C.c_double),
        ("v_ghost", C.c_double), ("disc", C.c_int), ("dtype", C.c_int),
        ("m_b", C.c_int), ("velocity_b", C.POINTER(C.c_double)), ("speed_axes", C.c_int),
        ("interp", C.c_int),
    ]


class SlRaOpts(C.Structure):
    _fields_ = [("coarse_stride", C.c_int), ("coarse_n", C.c_int * 3), ("C", C.c_double),
                ("M", C.c_double),
                ("q", C.c_double), ("delta_override", C.c_double), ("tol", C.c_double),
                ("max_sweeps", C.c_long), ("autotune", C.c_int), ("local_iters", C.c_int)]


class SlSolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_sweeps", C.c_long), ("want_policy", C.c_int),
                ("check_every", C.c_int), ("profile", C.c_int), ("autotune", C.c_int),
                ("local_iters", C.c_int)]


class SlStats(C.Structure):
    _fields_ = [("sweeps_max", C.c_long), ("sweeps_total", C.c_long), ("residual", C.c_double),
                ("node_control_updates", C.c_double), ("ms_ra", C.c_double),
                ("ms_fine", C.c_double), ("ms_total", C.c_double), ("n_subdomains", C.c_int),
                ("n_unreachable", C.c_int), ("set_fraction_max", C.c_double),
                ("ms_sweeps", C.c_double), ("sweep_launches", C.c_long), ("variant", C.c_int),
                ("mode", C.c_int), ("tile", C.c_int * 3), ("ra_sweeps_max", C.c_long)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["tile"] = tuple(self.tile)
        return d



def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Load libslhjb.so (raises if it is not built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built: run `python -m paper_1405_3521_amd.build`")
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER
        L.sl_status_string.argtypes = [C.c_int]
        L.sl_status_string.restype = C.c_char_p
        L.sl_abi_version.restype = C.c_int
        if L.sl_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{_LIB_PATH} has ABI {L.sl_abi_version()}, the binding "
                               f"expects {ABI_VERSION}: rebuild it")
        L.sl_tune_candidates.argtypes = [C.c_int, C.c_int]
        L.sl_tune_candidates.restype = C.c_int
        L.sl_solve_workspace_size.argtypes = [P(SlProblem)]
        L.sl_solve_workspace_size.restype = C.c_size_t
        L.sl_solve.argtypes = [P(SlProblem), P(SlSolveOpts), C.c_void_p, C.c_size_t, C.c_void_p,
                               C.c_void_p, P(SlStats), C.c_void_p]
        L.sl_solve.restype = C.c_int
        L.sl_solve_noalloc.argtypes = [P(SlProblem), P(SlSolveOpts), C.c_void_p, C.c_void_p,
                                       P(SlStats), C.c_void_p]
        L.sl_solve_noalloc.restype = C.c_int
        L.sl_isa_workspace_size.argtypes = [P(SlProblem), P(SlRaOpts)]
        L.sl_isa_workspace_size.restype = C.c_size_t
        L.sl_reconstruct.argtypes = [P(SlProblem), P(SlRaOpts), C.c_void_p, C.c_size_t,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, P(SlStats),
                                     C.c_void_p]
        L.sl_reconstruct.restype = C.c_int
        L.sl_refine_workspace_size.argtypes = [P(SlProblem), P(SlRaOpts), C.c_int]
        L.sl_refine_workspace_size.restype = C.c_size_t
        L.sl_refine_split.argtypes = [P(SlProblem), P(SlRaOpts), C.c_int, C.c_double, C.c_void_p,
                                      C.c_size_t, C.c_void_p, P(C.c_int), P(C.c_double),
                                      P(SlStats), C.c_void_p]
        L.sl_refine_split.restype = C.c_int
        L.sl_solve_isa.argtypes = [P(SlProblem), P(SlRaOpts), C.c_void_p, P(SlSolveOpts),
                                   C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, P(SlStats), C.c_void_p]
        L.sl_solve_isa.restype = C.c_int
        L.sl_isa.argtypes = [P(SlProblem), P(SlRaOpts), P(SlSolveOpts), C.c_void_p, C.c_size_t,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p, P(SlStats), C.c_void_p]
        L.sl_isa.restype = C.c_int
        L.sl_batched_workspace_size.argtypes = [C.c_int, P(SlProblem), P(SlRaOpts)]
        L.sl_batched_workspace_size.restype = C.c_size_t
        L.sl_solve_batched.argtypes = [C.c_int, P(SlProblem), P(SlRaOpts), P(SlSolveOpts),
                                       C.c_void_p, C.c_size_t, P(C.c_void_p), P(C.c_void_p),
                                       P(C.c_void_p), P(C.c_void_p), P(SlStats), P(SlStats),
                                       C.c_void_p]
        L.sl_solve_batched.restype = C.c_int
        L.sl_adjoint_workspace_size.argtypes = [P(SlProblem), C.c_int]
        L.sl_adjoint_workspace_size.restype = C.c_size_t
        L.sl_adjoint.argtypes = [P(SlProblem), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_double, C.c_long, C.c_int, C.c_void_p, C.c_size_t,
                                 P(SlStats), C.c_void_p]
        L.sl_adjoint.restype = C.c_int
        _LIB = L
    return _LIB


# ------------------------------------------------------------------ problem data
@dataclass
class DeviceProblem:
    """A problem whose node fields are device tensors (see include/slhjb.h)."""
    dim: int
    n: tuple
    lo: tuple
    hi: tuple
    velocity: np.ndarray            # host (m, dim) float64 (a game: the pursuer's a_k)
    target: "object"                # torch.int8 device tensor (N,)
    n_comp: int
    speed: Optional[object] = None  # torch tensor (N,) or, per axis, (N*dim,) of `dtype`, or None
    cost: Optional[object] = None
    g: Optional[object] = None
    drift: Optional[object] = None  # torch tensor (N*dim,) of `dtype`, node-major, or None
    lam: float = 1.0
    h: float = 0.0
    v_ghost: float = 1.0
    disc: str = "exp"               # "exp", "paper" or "kruzkov" (per-node exp(-h l); see slhjb.h)
    dtype: "object" = None          # torch.float32 / torch.float64
    velocity_b: Optional[np.ndarray] = None  # host (m_b, dim) float64: the evader's b_l (games)
    speed_axes: bool = False        # speed holds dim factors per node (node-major)
    interp: str = "q1"              # "q1" (cells) or "p1" (Kuhn simplices)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    @property
    def m(self) -> int:
        return int(self.velocity.shape[0])

    @property
    def step(self) -> float:
        return self.h if self.h > 0 else (self.hi[0] - self.lo[0]) / (self.n[0] - 1)


@dataclass
class RaOpts:
    coarse_stride: int = 1
    coarse_n: Optional[tuple] = None      # coarse nodes per axis (any counts); None -> stride
    C: float = 0.5
    M: float = 0.5
    q: float = 1.0
    delta_override: float = 0.0
    tol: float = 0.0
    max_sweeps: int = 10_000_000
    autotune: int = 0
    local_iters: int = 0      # coarse sweeps: 0 Jacobi; k > 0 block-asynchronous


@dataclass
class SolveOpts:
    tol: float = 0.0
    max_sweeps: int = 10_000_000
    want_policy: bool = False
    check_every: int = 0
    profile: bool = False
    autotune: int = 0
    local_iters: int = 0      # 0: Jacobi sweeps; k > 0: block-asynchronous (see sl_solve_opts)


def to_device(prob, dtype=None, device: str = "cuda:0") -> DeviceProblem:
    """Copy a host problem description (any object with the attributes of
    ``DeviceProblem``, fields as numpy arrays) to device tensors of ``dtype``."""
    import torch
    dtype = dtype or torch.float32

    def dev(a, dt):
        return None if a is None else torch.as_tensor(np.ascontiguousarray(a)).to(device=device, dtype=dt)

    sp = getattr(prob, "speed", None)
    axes = sp is not None and np.asarray(sp).ndim == 2
    vb = getattr(prob, "velocity_b", None)
    return DeviceProblem(
        dim=prob.dim, n=tuple(prob.n), lo=tuple(prob.lo), hi=tuple(prob.hi),
        velocity=np.ascontiguousarray(prob.velocity, dtype=np.float64),
        target=dev(prob.target, torch.int8), n_comp=int(prob.n_comp),
        speed=None if sp is None else dev(np.asarray(sp).reshape(-1), dtype),
        speed_axes=axes, cost=dev(getattr(prob, "cost", None), dtype),
        velocity_b=None if vb is None else np.ascontiguousarray(vb, dtype=np.float64),
        g=dev(getattr(prob, "g", None), dtype),
        drift=None if getattr(prob, "drift", None) is None
        else dev(np.asarray(prob.drift).reshape(-1), dtype),
        lam=float(prob.lam),
        h=float(getattr(prob, "step", 0.0) or prob.h), v_ghost=float(prob.v_ghost),
        disc=prob.disc, dtype=dtype, interp=getattr(prob, "interp", "q1"))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_tensor(t, dtype, numel, name):
    import torch
    if t is None:
        return
    if not t.is_cuda or t.dtype != dtype or t.numel() != numel or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous {dtype} device tensor with {numel} elements")


def _cproblem(p: DeviceProblem):
    import torch
    N = p.N
    _check_tensor(p.target, torch.int8, N, "target")
    for name in ("cost", "g"):
        _check_tensor(getattr(p, name), p.dtype, N, name)
    _check_tensor(p.speed, p.dtype, N * (p.dim if p.speed_axes else 1), "speed")
    _check_tensor(p.drift, p.dtype, N * p.dim, "drift")
    vel = np.ascontiguousarray(p.velocity, dtype=np.float64)
    if vel.ndim != 2 or vel.shape[1] != p.dim:
        raise ValueError("velocity must have shape (m, dim)")
    vb = None if p.velocity_b is None else np.ascontiguousarray(p.velocity_b, dtype=np.float64)
    if vb is not None and (vb.ndim != 2 or vb.shape[1] != p.dim):
        raise ValueError("velocity_b must have shape (m_b, dim)")
    cp = SlProblem()
    cp.dim = p.dim
    for d in range(3):
        cp.n[d] = int(p.n[d]) if d < p.dim else 1
        cp.lo[d] = float(p.lo[d]) if d < p.dim else 0.0
        cp.hi[d] = float(p.hi[d]) if d < p.dim else 1.0
    cp.m = vel.shape[0]
    cp.velocity = vel.ctypes.data_as(C.POINTER(C.c_double))
    cp.speed = _ptr(p.speed)
    cp.cost = _ptr(p.cost)
    cp.drift = _ptr(p.drift)
    cp.target = _ptr(p.target)
    cp.g = _ptr(p.g)
    cp.n_comp = p.n_comp
    cp.lambda_ = p.lam
    cp.h = p.step
    cp.v_ghost = p.v_ghost
    cp.disc = DISC[p.disc]
    cp.dtype = 0 if p.dtype == torch.float32 else 1
    cp.m_b = 0 if vb is None else vb.shape[0]
    cp.velocity_b = None if vb is None else vb.ctypes.data_as(C.POINTER(C.c_double))
    cp.speed_axes = 1 if p.speed_axes else 0
    cp.interp = INTERP[p.interp]
    return cp, (vel, vb)     # keep the host tables alive


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ra(o: RaOpts) -> SlRaOpts:
    cn = tuple(o.coarse_n or ()) + (0, 0, 0)
    return SlRaOpts(o.coarse_stride, (C.c_int * 3)(*[int(x) for x in cn[:3]]), o.C, o.M, o.q,
                    o.delta_override, o.tol, o.max_sweeps, int(o.autotune), int(o.local_iters))


def refine_split(p: DeviceProblem, ra: RaOpts, max_comp: int, frac_goal: float = 0.0,
                 workspace=None):
    """Recursive halving of the target components for balance (see sl_refine_split).
    Returns (target ids as a device int8 tensor, component count, the largest set
    fraction after each reconstruction, stats)."""
    import torch
    L = lib()
    cp, keep = _cproblem(p)
    dev = p.target.device
    rao = _ra(ra)
    ws_bytes = L.sl_refine_workspace_size(C.byref(cp), C.byref(rao), int(max_comp))
    if ws_bytes == 0:
        raise ValueError("invalid problem, reconstruction options or max_comp")
    ws = workspace if workspace is not None and workspace.numel() >= ws_bytes else _workspace(ws_bytes, dev)
    tid = torch.empty(p.N, dtype=torch.int8, device=dev)
    nc = C.c_int(0)
    fr = (C.c_double * (int(max_comp) - p.n_comp + 1))()
    st = SlStats()
    rc = L.sl_refine_split(C.byref(cp), C.byref(rao), int(max_comp), float(frac_goal), _ptr(ws),
                           ws.numel(), _ptr(tid), C.byref(nc), fr, C.byref(st), _stream())
    if rc < 0:
        raise SlError("sl_refine_split", rc)
    d = st.as_dict()
    d["converged"] = rc == SL_OK
    return tid, nc.value, list(fr)[:d["sweeps_max"]], d


def coarse_nodes(p, ra: RaOpts) -> tuple:
    """Nodes per axis of the coarse grid that ``ra`` describes for problem ``p``."""
    if ra.coarse_n:
        return tuple(int(ra.coarse_n[d]) for d in range(p.dim))
    return tuple((p.n[d] - 1) // ra.coarse_stride + 1 for d in range(p.dim))


def _so(o: SolveOpts) -> SlSolveOpts:
    return SlSolveOpts(o.tol, o.max_sweeps, int(bool(o.want_policy)), o.check_every,
                       int(bool(o.profile)), int(o.autotune), int(o.local_iters))


def _workspace(nbytes: int, device):
    import torch
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def solve_workspace_bytes(p: DeviceProblem) -> int:
    """Workspace bytes of ``solve`` (sl_solve_workspace_size)."""
    cp, keep = _cproblem(p)
    return int(lib().sl_solve_workspace_size(C.byref(cp)))


def isa_workspace_bytes(p: DeviceProblem, ra: RaOpts) -> int:
    """Workspace bytes of ``reconstruct`` / ``solve_isa`` / ``isa``."""
    cp, keep = _cproblem(p)
    return int(lib().sl_isa_workspace_size(C.byref(cp), C.byref(_ra(ra))))


def adjoint_workspace_bytes(p: DeviceProblem, n_sets: int) -> int:
    """Workspace bytes of ``adjoint`` over n_sets sets (1 for the global solve)."""
    cp, keep = _cproblem(p)
    return int(lib().sl_adjoint_workspace_size(C.byref(cp), int(n_sets)))


def solve(p: DeviceProblem, opts: SolveOpts = SolveOpts(), out=None, policy=None,
          workspace=None):
    """Global value iteration (no decomposition).  Returns (V, policy or None, stats)."""
    import torch
    L = lib()
    cp, keep = _cproblem(p)
    dev = p.target.device
    ws_bytes = L.sl_solve_workspace_size(C.byref(cp))
    if ws_bytes == 0:
        raise ValueError("invalid problem")
    ws = workspace if workspace is not None and workspace.numel() >= ws_bytes else _workspace(ws_bytes, dev)
    V = out if out is not None else torch.empty(p.N, dtype=p.dtype, device=dev)
    pol = policy
    if opts.want_policy and pol is None:
        pol = torch.full((p.N,), 255, dtype=torch.uint8, device=dev)
    st = SlStats()
    rc = L.sl_solve(C.byref(cp), C.byref(_so(opts)), _ptr(ws), ws.numel(), _ptr(V), _ptr(pol),
                    C.byref(st), _stream())
    if rc < 0:
        raise SlError("sl_solve", rc)
    d = st.as_dict()
    d["converged"] = rc == SL_OK
    return V, pol, d


def solve_noalloc(p: DeviceProblem, opts: SolveOpts = SolveOpts(), out=None, policy=None):
    """The global solve of ``solve`` through sl_solve_noalloc: the library takes its
    workspace from its static device scratch instead of a caller workspace (see
    slhjb.h for the size limit).  ``out`` and ``policy`` are the caller's output
    tensors (allocated here when None).  Returns (V, policy or None, stats)."""
    import torch
    L = lib()
    cp, keep = _cproblem(p)
    dev = p.target.device
    V = out if out is not None else torch.empty(p.N, dtype=p.dtype, device=dev)
    _check_tensor(V, p.dtype, p.N, "out")
    pol = policy
    if opts.want_policy and pol is None:
        pol = torch.full((p.N,), 255, dtype=torch.uint8, device=dev)
    st = SlStats()
    rc = L.sl_solve_noalloc(C.byref(cp), C.byref(_so(opts)), _ptr(V), _ptr(pol), C.byref(st),
                            _stream())
    if rc < 0:
        raise SlError("sl_solve_noalloc", rc)
    d = st.as_dict()
    d["converged"] = rc == SL_OK
    return V, pol, d


def reconstruct(p: DeviceProblem, ra: RaOpts, want_coarse: bool = False, workspace=None):
    """RA on the coarse grid + projection.  Returns (member, label, stats[, mK, lK])."""
    import torch
    L = lib()
    cp, keep = _cproblem(p)
    dev = p.target.device
    cra = _ra(ra)
    ws_bytes = L.sl_isa_workspace_size(C.byref(cp), C.byref(cra))
    if ws_bytes == 0:
        raise ValueError("invalid problem or RA options")
    ws = workspace if workspace is not None and workspace.numel() >= ws_bytes else _workspace(ws_bytes, dev)
    member = torch.empty(p.N, dtype=torch.uint8, device=dev)
    label = torch.empty(p.N, dtype=torch.uint8, device=dev)
    NK = int(np.prod(coarse_nodes(p, ra)))
    mK = torch.empty(NK, dtype=torch.uint8, device=dev) if want_coarse else None
    lK = torch.empty(NK, dtype=torch.uint8, device=dev) if want_coarse else None
    st = SlStats()
    rc = L.sl_reconstruct(C.byref(cp), C.byref(cra), _ptr(ws), ws.numel(), _ptr(member),
                          _ptr(label), _ptr(mK), _ptr(lK), C.byref(st), _stream())
    if rc < 0:
        raise SlError("sl_reconstruct", rc)
    d = st.as_dict()
    d["converged"] = rc == SL_OK
    if want_coarse:
        return member, label, d, mK, lK
    return member, label, d


def solve_isa(p: DeviceProblem, ra: RaOpts, member, opts: SolveOpts = SolveOpts(),
              want_owner: bool = True, want_sets: bool = False, workspace=None):
    """ISA steps 3-4 on given sets.  Returns (V, owner, policy, V_sets, stats)."""
    import torch
    L = lib()
    cp, keep = _cproblem(p)
    dev = p.target.device
    _check_tensor(member, torch.uint8, p.N, "member")
    cra = _ra(ra)
    ws_bytes = L.sl_isa_workspace_size(C.byref(cp), C.byref(cra))
    if ws_bytes == 0:
        raise ValueError("invalid problem or RA options")
    ws = workspace if workspace is not None and workspace.numel() >= ws_bytes else _workspace(ws_bytes, dev)
    V = torch.empty(p.N, dtype=p.dtype, device=dev)
    owner = torch.empty(p.N, dtype=torch.uint8, device=dev) if want_owner else None
    pol = (torch.full((p.n_comp * p.N,), 255, dtype=torch.uint8, device=dev)
           if opts.want_policy else None)
    Vs = torch.empty(p.n_comp * p.N, dtype=p.dtype, device=dev) if want_sets else None
    st = SlStats()
    rc = L.sl_solve_isa(C.byref(cp), C.byref(cra), _ptr(member), C.byref(_so(opts)), _ptr(ws),
                        ws.numel(), _ptr(V), _ptr(owner), _ptr(pol), _ptr(Vs), C.byref(st),
                        _stream())
    if rc < 0:
        raise SlError("sl_solve_isa", rc)
    d = st.as_dict()
    d["converged"] = rc == SL_OK
    return V, owner, pol, Vs, d


def isa(p: DeviceProblem, ra: RaOpts, opts: SolveOpts = SolveOpts(), want_sets: bool = False,
        workspace=None):
    """The whole independent-sets algorithm in one library call (sl_isa):
    reconstruct, then solve the sets.  Returns (V, owner, member, label, policy,
    V_sets, stats); stats are the sets' solves' with ``ms_ra`` and
    ``ra_sweeps_max`` of the reconstruction."""
    import torch
    L = lib()
    cp, keep = _cproblem(p)
    dev = p.target.device
    cra = _ra(ra)
    ws_bytes = L.sl_isa_workspace_size(C.byref(cp), C.byref(cra))
    if ws_bytes == 0:
        raise ValueError("invalid problem or RA options")
    ws = workspace if workspace is not None and workspace.numel() >= ws_bytes else _workspace(ws_bytes, dev)
    V = torch.empty(p.N, dtype=p.dtype, device=dev)
    owner = torch.empty(p.N, dtype=torch.uint8, device=dev)
    member = torch.empty(p.N, dtype=torch.uint8, device=dev)
    label = torch.empty(p.N, dtype=torch.uint8, device=dev)
    pol = (torch.full((p.n_comp * p.N,), 255, dtype=torch.uint8, device=dev)
           if opts.want_policy else None)
    Vs = torch.empty(p.n_comp * p.N, dtype=p.dtype, device=dev) if want_sets else None
    st = SlStats()
    rc = L.sl_isa(C.byref(cp), C.byref(cra), C.byref(_so(opts)), _ptr(ws), ws.numel(), _ptr(V),
                  _ptr(owner), _ptr(member), _ptr(label), _ptr(pol), _ptr(Vs), C.byref(st),
                  _stream())
    if rc < 0:
        raise SlError("sl_isa", rc)
    d = st.as_dict()
    d["converged"] = rc == SL_OK
    return V, owner, member, label, pol, Vs, d


class IsaSolver:
    """``isa`` on one problem with its arguments marshalled once and its outputs
    and workspace kept across calls: a loop that solves the same problem (or new
    values in the same field tensors) pays only the library call.  ``solve``
    returns (V, owner, member, label, policy, V_sets, stats) like ``isa``; the
    tensors are this object's and are overwritten by the next call."""

    def __init__(self, p: DeviceProblem, ra: RaOpts, want_sets: bool = False,
                 want_policy: bool = False):
        import torch
        L = lib()
        self.p = p
        self.cp, self._keep = _cproblem(p)
        self.cra = _ra(ra)
        dev = p.target.device
        ws_bytes = L.sl_isa_workspace_size(C.byref(self.cp), C.byref(self.cra))
        if ws_bytes == 0:
            raise ValueError("invalid problem or RA options")
        self.ws = _workspace(ws_bytes, dev)
        self.V = torch.empty(p.N, dtype=p.dtype, device=dev)
        self.owner = torch.empty(p.N, dtype=torch.uint8, device=dev)
        self.member = torch.empty(p.N, dtype=torch.uint8, device=dev)
        self.label = torch.empty(p.N, dtype=torch.uint8, device=dev)
        self.pol = (torch.full((p.n_comp * p.N,), 255, dtype=torch.uint8, device=dev)
                    if want_policy else None)
        self.Vs = torch.empty(p.n_comp * p.N, dtype=p.dtype, device=dev) if want_sets else None
        self._args = [_ptr(self.ws), self.ws.numel(), _ptr(self.V), _ptr(self.owner),
                      _ptr(self.member), _ptr(self.label), _ptr(self.pol), _ptr(self.Vs)]
        self.st = SlStats()

    def solve(self, opts: SolveOpts = SolveOpts()):
        if opts.want_policy and self.pol is None:
            raise ValueError("IsaSolver built without want_policy")
        rc = lib().sl_isa(C.byref(self.cp), C.byref(self.cra), C.byref(_so(opts)), *self._args,
                          C.byref(self.st), _stream())
        if rc < 0:
            raise SlError("sl_isa", rc)
        d = self.st.as_dict()
        d["converged"] = rc == SL_OK
        return self.V, self.owner, self.member, self.label, self.pol, self.Vs, d


def adjoint(p: DeviceProblem, policy, dLdV, member=None, owner=None, tol: float = None,
            max_iters: int = 100_000, local_iters: int = 0, workspace=None):
    """dL/dl of a loss with gradient dL/dV, the forward's controls frozen.

    ``tol``: stop when the adjoint state changes by at most tol (plus the
    library's rounding allowance, 16 eps max|lambda|) in one iteration; default 0.
    A negative tol is relative: |tol| * max |dLdV|, rounded down to a power of two.
    ``local_iters``: 0 Jacobi iteration; k > 0 block-asynchronous tiles (2D).

    ``policy``: from the forward call (``solve``: N entries; ``solve_isa``:
    n_comp*N).  With ``member`` (sets) ``owner`` routes dL/dV to the owning set.
    Returns (dLdl, stats)."""
    import torch
    L = lib()
    cp, keep = _cproblem(p)
    dev = p.target.device
    n_sets = p.n_comp if member is not None else 1
    _check_tensor(policy, torch.uint8, n_sets * p.N, "policy")
    _check_tensor(dLdV, p.dtype, p.N, "dLdV")
    if member is not None:
        _check_tensor(member, torch.uint8, p.N, "member")
        _check_tensor(owner, torch.uint8, p.N, "owner")
    if tol is None:
        tol = 0.0
    ws_bytes = L.sl_adjoint_workspace_size(C.byref(cp), n_sets)
    if ws_bytes == 0:
        raise ValueError("invalid problem")
    ws = workspace if workspace is not None and workspace.numel() >= ws_bytes else _workspace(ws_bytes, dev)
    out = torch.empty(p.N, dtype=p.dtype, device=dev)
    st = SlStats()
    rc = L.sl_adjoint(C.byref(cp), _ptr(member), _ptr(owner), _ptr(policy), _ptr(dLdV),
                      _ptr(out), float(tol), int(max_iters), int(local_iters), _ptr(ws),
                      ws.numel(), C.byref(st),
                      _stream())
    if rc < 0:
        raise SlError("sl_adjoint", rc)
    d = st.as_dict()
    d["converged"] = rc == SL_OK
    return out, d


class BatchedSolver:
    """A batch marshalled once for repeated calls of sl_solve_batched: the problem
    and option structs, the output tensors (V, member, label, owner per problem),
    their pointer arrays and the workspace are built here; ``solve`` only makes
    the call.  The problems' device fields must stay alive and unchanged in shape
    while the solver is used (their values may change between calls)."""

    def __init__(self, problems, ras, want_owner: bool = True, workspace=None):
        import torch
        L = lib()
        n = len(problems)
        if n == 0 or len(ras) != n:
            raise ValueError("need one RaOpts per problem")
        cps, self._keep = [], []
        for p in problems:
            cp, k = _cproblem(p)
            cps.append(cp)
            self._keep.append(k)
        self.n = n
        self.arr = (SlProblem * n)(*cps)
        self.rarr = (SlRaOpts * n)(*[_ra(r) for r in ras])
        dev = problems[0].target.device
        ws_bytes = L.sl_batched_workspace_size(n, self.arr, self.rarr)
        if ws_bytes == 0:
            raise ValueError("invalid batch (problems must share dim and dtype)")
        self.ws = (workspace if workspace is not None and workspace.numel() >= ws_bytes
                   else _workspace(ws_bytes, dev))
        self.V = [torch.empty(p.N, dtype=p.dtype, device=dev) for p in problems]
        self.member = [torch.empty(p.N, dtype=torch.uint8, device=dev) for p in problems]
        self.label = [torch.empty(p.N, dtype=torch.uint8, device=dev) for p in problems]
        self.owner = ([torch.empty(p.N, dtype=torch.uint8, device=dev) for p in problems]
                      if want_owner else None)
        ptrs = lambda ts: (C.c_void_p * n)(*[t.data_ptr() for t in ts])
        self._pV, self._pm, self._pl = ptrs(self.V), ptrs(self.member), ptrs(self.label)
        self._po = ptrs(self.owner) if self.owner else None
        self.per = (SlStats * n)()
        self.tot = SlStats()

    def solve(self, opts: SolveOpts = SolveOpts()):
        """One batched solve into the solver's output tensors.  Returns (V list,
        member list, label list, owner list, total stats); per-problem stats are
        in ``per_problem()``."""
        rc = lib().sl_solve_batched(self.n, self.arr, self.rarr, C.byref(_so(opts)),
                                    _ptr(self.ws), self.ws.numel(), self._pV, self._pm,
                                    self._pl, self._po, self.per, C.byref(self.tot), _stream())
        if rc < 0:
            raise SlError("sl_solve_batched", rc)
        t = self.tot.as_dict()
        t["converged"] = rc == SL_OK
        return self.V, self.member, self.label, self.owner, t

    def per_problem(self):
        return [x.as_dict() for x in self.per]


def solve_batched(problems, ras, opts: SolveOpts = SolveOpts(), want_owner: bool = True,
                  workspace=None):
    """The independent-sets algorithm for many problems at once (one launch per
    step for all of them).  Returns (V list, member list, label list, owner list,
    per-problem stats list, total stats)."""
    b = BatchedSolver(problems, ras, want_owner, workspace)
    Vs, mem, lab, own, t = b.solve(opts)
    return Vs, mem, lab, own, b.per_problem(), t


from .autograd import HJBSolve  # noqa: E402
