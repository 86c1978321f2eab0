"""The C-ABI library without a GPU: it loads, exports every function the header
declares, and rejects bad arguments on the host before any device work."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1405_3521_amd as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slhjb.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_][\w]*\s*\**\s*(sl_\w+)\s*\(", src, re.M)
    return sorted(set(names))


def test_library_exports_every_declared_function():
    L = S.lib()
    names = declared_functions()
    assert len(names) >= 7
    for n in names:
        assert hasattr(L, n), f"{n} declared in slhjb.h but not exported"


def test_abi_version_matches_header():
    m = re.search(r"#define SLHJB_ABI_VERSION (\d+)", open(HEADER).read())
    assert S.lib().sl_abi_version() == int(m.group(1))


def test_status_strings():
    L = S.lib()
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert L.sl_status_string(code)
    assert b"unknown" in L.sl_status_string(42)


def _problem(**kw):
    vel = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]])
    p = S.SlProblem()
    p.dim = 2
    p.n[0], p.n[1], p.n[2] = 9, 9, 1
    for d in range(3):
        p.lo[d], p.hi[d] = -1.0, 1.0
    p.m = 4
    p.velocity = vel.ctypes.data_as(C.POINTER(C.c_double))
    p.target = C.c_void_p(0x1000)          # never dereferenced on the host
    p.n_comp = 1
    p.lambda_ = 1.0
    p.h = 0.25
    p.v_ghost = 1.0
    p.disc = 0
    p.dtype = 0
    for k, v in kw.items():
        setattr(p, k, v)
    return p, vel


def test_workspace_query_rejects_invalid_problems():
    L = S.lib()
    assert L.sl_solve_workspace_size(None) == 0
    good, keep = _problem()
    assert L.sl_solve_workspace_size(C.byref(good)) > 0
    for bad in (dict(dim=4), dict(m=0), dict(m=300), dict(n_comp=0), dict(n_comp=9),
                dict(lambda_=0.0), dict(h=-1.0), dict(disc=5), dict(dtype=7),
                dict(v_ghost=float("nan"))):
        p, keep = _problem(**bad)
        assert L.sl_solve_workspace_size(C.byref(p)) == 0, bad
    p, keep = _problem()
    p.n[0] = 2
    assert L.sl_solve_workspace_size(C.byref(p)) == 0


def test_solve_argument_errors_before_device_work():
    L = S.lib()
    p, keep = _problem()
    opts = S.SlSolveOpts(0.0, 100, 0, 0, 0)
    st = S.SlStats()
    buf = C.create_string_buffer(64)
    # null problem / options / outputs
    assert L.sl_solve(None, C.byref(opts), buf, 64, buf, None, C.byref(st), None) == -1
    assert L.sl_solve(C.byref(p), None, buf, 64, buf, None, C.byref(st), None) == -1
    assert L.sl_solve(C.byref(p), C.byref(opts), buf, 64, None, None, C.byref(st), None) == -1
    # unsupported dimension
    q, keep2 = _problem(dim=1)
    assert L.sl_solve(C.byref(q), C.byref(opts), buf, 64, buf, None, C.byref(st), None) == -3
    # bad options
    bad = S.SlSolveOpts(-1.0, 100, 0, 0, 0)
    assert L.sl_solve(C.byref(p), C.byref(bad), buf, 64, buf, None, C.byref(st), None) == -1
    bad = S.SlSolveOpts(0.0, 0, 0, 0, 0)
    assert L.sl_solve(C.byref(p), C.byref(bad), buf, 64, buf, None, C.byref(st), None) == -1
    for li in (-1, 1025):          # local iterations out of [0, 1024]
        bad = S.SlSolveOpts(0.0, 100, 0, 0, 0, 0, li)
        assert L.sl_solve(C.byref(p), C.byref(bad), buf, 64, buf, None, C.byref(st), None) == -1
    ok = S.SlSolveOpts(0.0, 100, 0, 0, 0, 0, 1024)
    assert L.sl_solve(C.byref(p), C.byref(ok), buf, 64, buf, None, C.byref(st), None) == -5
    # workspace too small
    assert L.sl_solve(C.byref(p), C.byref(opts), buf, 64, buf, None, C.byref(st), None) == -5


def test_policy_byte_holds_at_most_255_controls():
    """A policy byte marks target and non-member nodes with 255, so a policy output
    (or an adjoint's policy input) with m = 256 controls is refused on the host;
    m = 255 passes the check (and then fails on the too-small workspace)."""
    L = S.lib()
    st = S.SlStats()
    buf = C.create_string_buffer(64)
    want = S.SlSolveOpts(0.0, 100, 1, 0, 0, 0, 0)
    ra = S.SlRaOpts(2, (C.c_int * 3)(0, 0, 0), 0.5, 0.5, 1.0, 0.0, 0.0, 1000)
    for m, code in ((256, -3), (255, -5)):
        vel = np.stack([np.cos(np.arange(m)), np.sin(np.arange(m))], axis=1)
        p, keep = _problem(m=m, velocity=vel.ctypes.data_as(C.POINTER(C.c_double)))
        assert L.sl_solve(C.byref(p), C.byref(want), buf, 64, buf, buf, C.byref(st), None) == code
        assert L.sl_solve_isa(C.byref(p), C.byref(ra), buf, C.byref(want), buf, 64, buf, None,
                              buf, None, C.byref(st), None) == code
        assert L.sl_adjoint(C.byref(p), None, None, buf, buf, buf, 0.0, 10, 0, buf, 64,
                            C.byref(st), None) == code
        # without a policy buffer the control count may reach SL_MAX_CONTROLS
        nopol = S.SlSolveOpts(0.0, 100, 0, 0, 0, 0, 0)
        assert L.sl_solve(C.byref(p), C.byref(nopol), buf, 64, buf, None, C.byref(st), None) == -5


def test_noalloc_entry_point_host_checks():
    """sl_solve_noalloc refuses, before any device work: problems whose workspace
    exceeds the static scratch (SL_ERR_SCRATCH), the options that time with HIP
    events (autotune > 0, profile), and everything sl_solve refuses."""
    L = S.lib()
    st = S.SlStats()
    buf = C.create_string_buffer(64)
    limit = 32 << 20
    m = re.search(r"#define SL_NOALLOC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)",
                  open(HEADER).read())
    assert (int(m.group(1)) << int(m.group(2))) == limit
    opts = S.SlSolveOpts(0.0, 100, 0, 0, 0, 0, 0)
    big, keep = _problem()
    big.n[0], big.n[1] = 2049, 2049
    assert L.sl_solve_workspace_size(C.byref(big)) > limit
    assert L.sl_solve_noalloc(C.byref(big), C.byref(opts), buf, None, C.byref(st), None) == -6
    assert b"static scratch" in L.sl_status_string(-6)
    small, keep2 = _problem()
    assert L.sl_solve_workspace_size(C.byref(small)) <= limit
    for bad in (S.SlSolveOpts(0.0, 100, 0, 0, 0, 1, 0), S.SlSolveOpts(0.0, 100, 0, 0, 1, 0, 0),
                S.SlSolveOpts(-1.0, 100, 0, 0, 0, 0, 0)):
        assert L.sl_solve_noalloc(C.byref(small), C.byref(bad), buf, None, C.byref(st),
                                  None) == -1
    assert L.sl_solve_noalloc(C.byref(small), C.byref(opts), None, None, C.byref(st), None) == -1
    assert L.sl_solve_noalloc(None, C.byref(opts), buf, None, C.byref(st), None) == -1
    q, keep3 = _problem(dim=1)
    assert L.sl_solve_noalloc(C.byref(q), C.byref(opts), buf, None, C.byref(st), None) == -3


def test_reconstruction_argument_errors():
    L = S.lib()
    p, keep = _problem()
    st = S.SlStats()
    buf = C.create_string_buffer(64)
    nested = lambda s: S.SlRaOpts(s, (C.c_int * 3)(0, 0, 0), 0.5, 0.5, 1.0, 0.0, 0.0, 1000)
    counts = lambda a, b: S.SlRaOpts(1, (C.c_int * 3)(a, b, 0), 0.5, 0.5, 1.0, 0.0, 0.0, 1000)
    ra = nested(3)                                         # 3 does not divide n-1 = 8
    assert L.sl_isa_workspace_size(C.byref(p), C.byref(ra)) == 0
    assert L.sl_reconstruct(C.byref(p), C.byref(ra), buf, 64, buf, buf, None, None,
                            C.byref(st), None) == -1
    ra = nested(2)
    assert L.sl_isa_workspace_size(C.byref(p), C.byref(ra)) > 0
    assert L.sl_reconstruct(C.byref(p), C.byref(ra), buf, 64, buf, buf, None, None,
                            C.byref(st), None) == -5
    ra = nested(4)                                         # coarse grid of 3 nodes: allowed
    assert L.sl_isa_workspace_size(C.byref(p), C.byref(ra)) > 0
    ra = nested(8)                                         # coarse grid of 2 nodes: too coarse
    assert L.sl_isa_workspace_size(C.byref(p), C.byref(ra)) == 0
    # node counts: any 3 <= nK_d <= n_d (here n = 9), nested or not
    assert L.sl_isa_workspace_size(C.byref(p), C.byref(counts(4, 6))) > 0
    assert L.sl_isa_workspace_size(C.byref(p), C.byref(counts(9, 3))) > 0
    assert L.sl_isa_workspace_size(C.byref(p), C.byref(counts(2, 5))) == 0
    assert L.sl_isa_workspace_size(C.byref(p), C.byref(counts(5, 10))) == 0
    assert L.sl_reconstruct(C.byref(p), C.byref(counts(5, 0)), buf, 64, buf, buf, None, None,
                            C.byref(st), None) == -1


def test_single_call_isa_argument_errors():
    """sl_isa refuses on the host what sl_reconstruct and sl_solve_isa refuse:
    missing outputs, an invalid RA grid, bad solve options, a too small
    workspace; a negative adjoint tolerance is a relative one, not an error."""
    L = S.lib()
    p, keep = _problem()
    st = S.SlStats()
    buf = C.create_string_buffer(64)
    opts = S.SlSolveOpts(0.0, 100, 0, 0, 0, 0, 0)
    ra = S.SlRaOpts(2, (C.c_int * 3)(0, 0, 0), 0.5, 0.5, 1.0, 0.0, 0.0, 1000)
    args = lambda **kw: [C.byref(kw.get("p", p)), C.byref(kw.get("ra", ra)),
                         C.byref(kw.get("o", opts)), buf, kw.get("ws", 64),
                         kw.get("V", buf), None, kw.get("member", buf), kw.get("label", buf),
                         None, None, C.byref(st), None]
    assert L.sl_isa(*args()) == -5                                  # workspace too small
    assert L.sl_isa(*args(member=None)) == -1
    assert L.sl_isa(*args(label=None)) == -1
    assert L.sl_isa(*args(V=None)) == -1
    bad_ra = S.SlRaOpts(3, (C.c_int * 3)(0, 0, 0), 0.5, 0.5, 1.0, 0.0, 0.0, 1000)
    assert L.sl_isa(*args(ra=bad_ra)) == -1
    assert L.sl_isa(*args(o=S.SlSolveOpts(-1.0, 100, 0, 0, 0, 0, 0))) == -1
    q, keep2 = _problem(dim=1)
    assert L.sl_isa(*args(p=q)) == -3
    # sl_adjoint: a negative (relative) tolerance passes the checks, a non-finite
    # one does not (both then meet the too-small workspace or the argument error)
    assert L.sl_adjoint(C.byref(p), None, None, buf, buf, buf, -1e-6, 10, 0, buf, 64,
                        C.byref(st), None) == -5
    assert L.sl_adjoint(C.byref(p), None, None, buf, buf, buf, float("nan"), 10, 0, buf, 64,
                        C.byref(st), None) == -1


def test_binding_raises_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(S, "_LIB", None)
    monkeypatch.setattr(S, "_LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        S.lib()


def test_drift_accepted_by_every_entry_point():
    """Control-affine dynamics with a drift: sl_solve / sl_reconstruct / sl_solve_isa,
    the batch and the adjoint size a workspace with room for the scaled drift; the
    adjoint passes its argument checks and stops at the workspace size (-5) before
    any device work."""
    L = S.lib()
    p, keep = _problem(drift=C.c_void_p(0x2000))
    q, keep2 = _problem()
    assert L.sl_solve_workspace_size(C.byref(p)) > L.sl_solve_workspace_size(C.byref(q))
    ra = S.SlRaOpts(2, (C.c_int * 3)(0, 0, 0), 0.5, 0.5, 1.0, 0.0, 0.0, 1000)
    assert L.sl_isa_workspace_size(C.byref(p), C.byref(ra)) > 0
    assert L.sl_batched_workspace_size(1, C.byref(p), C.byref(ra)) > L.sl_batched_workspace_size(
        1, C.byref(q), C.byref(ra))
    assert L.sl_adjoint_workspace_size(C.byref(p), 1) > L.sl_adjoint_workspace_size(
        C.byref(q), 1)
    buf = C.create_string_buffer(64)
    st = S.SlStats()
    assert L.sl_adjoint(C.byref(p), None, None, buf, buf, buf, 0.0, 10, 0, buf, 64,
                        C.byref(st), None) == -5


def test_game_and_axis_speed_fields_are_validated():
    """Differential games (m_b evader choices) and per-axis speed factors: the
    workspace queries size a game's larger displacement table and reject malformed
    fields; the batch takes both; the adjoint takes axis factors (and stops at the
    workspace size, -5) but not games, which, like a game with a policy output,
    report SL_ERR_UNSUPPORTED (-3) before any device work."""
    L = S.lib()
    vb = 0.5 * np.stack([np.cos(np.arange(20)), np.sin(np.arange(20))], axis=1)
    vbp = vb.ctypes.data_as(C.POINTER(C.c_double))
    game, k1 = _problem(m_b=20, velocity_b=vbp)           # 80 table rows
    ctrl, k2 = _problem()
    assert L.sl_solve_workspace_size(C.byref(game)) > L.sl_solve_workspace_size(C.byref(ctrl))
    for bad in (dict(m_b=3), dict(velocity_b=vbp), dict(m_b=-1, velocity_b=vbp),
                dict(m_b=257, velocity_b=vbp), dict(speed_axes=1), dict(speed_axes=2)):
        p, k = _problem(**bad)
        assert L.sl_solve_workspace_size(C.byref(p)) == 0, bad
    va = np.zeros((64, 2))
    vbig = np.zeros((65, 2))
    wide, k3 = _problem(m=64, velocity=va.ctypes.data_as(C.POINTER(C.c_double)), m_b=65,
                        velocity_b=vbig.ctypes.data_as(C.POINTER(C.c_double)))
    assert L.sl_solve_workspace_size(C.byref(wide)) == 0      # 64 * 65 rows > SL_MAX_TABLE
    wide.m_b = 64
    assert L.sl_solve_workspace_size(C.byref(wide)) > 0       # 64 * 64 = SL_MAX_TABLE
    nan = np.array([[np.nan, 0.0]])
    pn, k4 = _problem(m_b=1, velocity_b=nan.ctypes.data_as(C.POINTER(C.c_double)))
    assert L.sl_solve_workspace_size(C.byref(pn)) == 0
    axes, k5 = _problem(speed_axes=1, speed=C.c_void_p(0x3000))
    assert L.sl_solve_workspace_size(C.byref(axes)) > 0
    ra = S.SlRaOpts(2, (C.c_int * 3)(0, 0, 0), 0.5, 0.5, 1.0, 0.0, 0.0, 1000)
    assert L.sl_isa_workspace_size(C.byref(game), C.byref(ra)) > 0
    assert L.sl_batched_workspace_size(1, C.byref(game), C.byref(ra)) > 0     # games batch
    assert L.sl_batched_workspace_size(1, C.byref(axes), C.byref(ra)) > 0     # and axis factors
    for p, rc in ((game, -3), (axes, -5)):
        buf = C.create_string_buffer(64)
        st = S.SlStats()
        assert L.sl_adjoint(C.byref(p), None, None, buf, buf, buf, 0.0, 10, 0, buf, 64,
                            C.byref(st), None) == rc
    buf = C.create_string_buffer(64)
    o = S.SlSolveOpts()
    o.tol, o.max_sweeps, o.want_policy = 0.0, 10, 1
    st = S.SlStats()
    assert L.sl_solve(C.byref(game), C.byref(o), buf, 64, buf, buf, C.byref(st), None) == -3
    assert L.sl_solve_isa(C.byref(game), C.byref(ra), buf, C.byref(o), buf, 64, buf, None, buf,
                          None, C.byref(st), None) == -3


def test_refine_split_argument_checks():
    L = S.lib()
    p, keep = _problem()
    ra = S.SlRaOpts(2, (C.c_int * 3)(0, 0, 0), 0.5, 0.5, 1.0, 0.0, 0.0, 1000)
    assert L.sl_refine_workspace_size(C.byref(p), C.byref(ra), 4) > L.sl_isa_workspace_size(
        C.byref(p), C.byref(ra))
    assert L.sl_refine_workspace_size(C.byref(p), C.byref(ra), 0) == 0     # below n_comp
    assert L.sl_refine_workspace_size(C.byref(p), C.byref(ra), 9) == 0     # above SL_MAX_COMP
    buf = C.create_string_buffer(64)
    nc = C.c_int(0)
    st = S.SlStats()
    assert L.sl_refine_split(C.byref(p), C.byref(ra), 4, 1.5, buf, 64, buf, C.byref(nc), None,
                             C.byref(st), None) == -1                        # goal outside [0, 1]
    assert L.sl_refine_split(C.byref(p), C.byref(ra), 4, 0.0, buf, 64, None, C.byref(nc), None,
                             C.byref(st), None) == -1
    assert L.sl_refine_split(C.byref(p), C.byref(ra), 4, 0.0, buf, 64, buf, C.byref(nc), None,
                             C.byref(st), None) == -5                        # workspace too small


def test_kruzkov_form_accepted_by_solves_and_batch_rejected_by_adjoint():
    L = S.lib()
    p, keep = _problem(disc=2, cost=C.c_void_p(0x4000))
    q, keep2 = _problem(cost=C.c_void_p(0x4000))
    # one more per-node field (the discount)
    assert L.sl_solve_workspace_size(C.byref(p)) > L.sl_solve_workspace_size(C.byref(q))
    bad, keep3 = _problem(disc=3)
    assert L.sl_solve_workspace_size(C.byref(bad)) == 0
    ra = S.SlRaOpts(2, (C.c_int * 3)(0, 0, 0), 0.5, 0.5, 1.0, 0.0, 0.0, 1000)
    assert L.sl_isa_workspace_size(C.byref(p), C.byref(ra)) > 0
    assert L.sl_batched_workspace_size(1, C.byref(p), C.byref(ra)) > L.sl_batched_workspace_size(
        1, C.byref(q), C.byref(ra))
    buf = C.create_string_buffer(64)
    st = S.SlStats()
    assert L.sl_adjoint(C.byref(p), None, None, buf, buf, buf, 0.0, 10, 0, buf, 64,
                        C.byref(st), None) == -3


def test_p1_interpolation_field_is_validated():
    """interp: Q1 (0) or P1 (1).  P1 is sized by the solves and the
    reconstruction in 2D and 3D; other values are refused by every workspace query,
    the batch takes P1 but not a mix of P1 and Q1, and the adjoint takes it (and
    stops at the workspace size, -5, before any device work)."""
    L = S.lib()
    p, k1 = _problem(interp=1)
    q, k2 = _problem()
    assert L.sl_solve_workspace_size(C.byref(p)) == L.sl_solve_workspace_size(C.byref(q)) > 0
    ra = S.SlRaOpts(2, (C.c_int * 3)(0, 0, 0), 0.5, 0.5, 1.0, 0.0, 0.0, 1000)
    assert L.sl_isa_workspace_size(C.byref(p), C.byref(ra)) > 0
    assert L.sl_batched_workspace_size(1, C.byref(p), C.byref(ra)) > 0
    pair = (S.SlProblem * 2)(p, q)                 # one interpolation per batch
    ras = (S.SlRaOpts * 2)(ra, ra)
    assert L.sl_batched_workspace_size(2, pair, ras) == 0
    bad, k3 = _problem(interp=2)
    assert L.sl_solve_workspace_size(C.byref(bad)) == 0
    v3 = np.eye(3)
    p3, k4 = _problem(interp=1, dim=3, m=3, velocity=v3.ctypes.data_as(C.POINTER(C.c_double)))
    p3.n[2] = 9
    assert L.sl_solve_workspace_size(C.byref(p3)) > 0
    p3.interp = 3
    assert L.sl_solve_workspace_size(C.byref(p3)) == 0
    buf = C.create_string_buffer(64)
    st = S.SlStats()
    assert L.sl_adjoint(C.byref(p), None, None, buf, buf, buf, 0.0, 10, 0, buf, 64,
                        C.byref(st), None) == -5
