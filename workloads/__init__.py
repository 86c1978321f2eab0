"""Seeded synthetic problem data for the semi-Lagrangian HJB solver.

This module only *builds problem data*: grids, discrete control tables, speed and
cost fields, target masks, observation sets.  It holds none of the scheme's
arithmetic (no foot computation, no interpolation, no discounting, no iteration).
Both the FP64 oracle (``oracle/``) and the HIP library read the arrays it returns,
so a generator detail can never break parity between them.

Conventions
-----------
* Grids are uniform boxes, ``n[d]`` nodes per axis, node ``i`` at ``lo + i*dx`` with
  ``dx = (hi - lo)/(n - 1)``.  Flat arrays are row-major with x fastest:
  ``j = i0 + n0*(i1 + n1*i2)``.
* Dynamics are ``f(x, a_k) = c(x) * b_k``: a positive speed field ``c`` times a
  tabulated velocity ``b_k`` per discrete control (``velocity``, shape ``(m, d)``),
  plus an optional drift.  A differential game adds the evader's table
  (``velocity_b``, shape ``(mb, d)``): ``f(x, a_k, b_l) = drift(x) + S(x)(a_k - b_l)``
  with ``S`` the speed times the identity, or ``diag(speed[j, :])`` when the speed
  has one factor per axis (shape ``(N, d)``).
* ``target[j] = -1`` marks a free node, ``k >= 0`` a node of target component ``k``.
* Every floating field is rounded to float32 and then stored as float64, so the
  FP32 GPU path and the FP64 oracle see bit-identical inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "Problem", "grid_axes", "node_coords", "controls_2d", "controls_3d_fibonacci",
    "spd_matrix", "gaussian_field", "separated_centres", "ball_targets", "coarse_stride",
    "coarse_nodes_for",
    "c1_eikonal", "c2_multitarget", "c3_aniso3d", "c4_batch", "c5_adjoint",
    "strip_problem", "box_distance_problem", "vdp_problem", "obs_nodes",
    "circle_controls", "pursuit_evasion_problem", "strip_game_problem", "kruzkov_problem",
]


@dataclass
class Problem:
    """Data of one exit-time problem on a uniform box grid (see the module doc)."""
    name: str
    dim: int
    n: tuple
    lo: tuple
    hi: tuple
    velocity: np.ndarray                 # (m, dim) float64, f(x,a_k) = c(x) * velocity[k]
    target: np.ndarray                   # (N,) int8, -1 free, k >= 0 component k
    n_comp: int
    speed: Optional[np.ndarray] = None   # (N,) or per axis (N, dim), float32-representable; None -> 1
    cost: Optional[np.ndarray] = None    # (N,) running cost l(x) > 0; None -> 1
    g: Optional[np.ndarray] = None       # (N,) exit cost on target nodes; None -> 0
    drift: Optional[np.ndarray] = None   # (N, dim) drift b(x), f = b(x) + c(x)*velocity; None -> 0
    lam: float = 1.0
    h: float = 0.0                       # 0 -> h = dx (first axis)
    v_ghost: float = 1.0
    disc: str = "exp"                    # "exp": beta=e^{-lam h}; "paper": beta=1/(1+lam h); "kruzkov": beta_j=e^{-h l_j}
    coarse_stride: int = 1
    coarse_n: Optional[tuple] = None     # coarse nodes per axis; None -> every coarse_stride-th node
    ra_C: float = 0.5                    # RA threshold 2 (C dx^q + M dx); these defaults
    ra_M: float = 0.5                    # give delta = 2 dx_K (the benchmark workloads take
                                         # C = M = q = 1, delta = 4 dx_K)
    ra_q: float = 1.0
    ra_tol: float = 0.0                  # coarse stopping tolerance (0: until nothing changes)
    velocity_b: Optional[np.ndarray] = None  # (mb, dim) evader's table (games); None -> control problem
    interp: str = "q1"                   # "q1": Q1 on cells; "p1": P1 on the Kuhn simplices of each cell
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    @property
    def m(self) -> int:
        return int(self.velocity.shape[0])

    @property
    def dx(self) -> tuple:
        return tuple((self.hi[d] - self.lo[d]) / (self.n[d] - 1) for d in range(self.dim))

    @property
    def step(self) -> float:
        return self.h if self.h > 0 else self.dx[0]

    def shape(self) -> tuple:
        """numpy shape of a node field (slowest axis first)."""
        return tuple(reversed(self.n))

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


# ----------------------------------------------------------------------------- grids
def grid_axes(n: Sequence[int], lo: Sequence[float], hi: Sequence[float]) -> List[np.ndarray]:
    """1D node coordinate arrays per axis."""
    return [lo[d] + (hi[d] - lo[d]) / (n[d] - 1) * np.arange(n[d], dtype=np.float64)
            for d in range(len(n))]


def node_coords(n, lo, hi) -> np.ndarray:
    """(N, d) node coordinates in flat (x fastest) order."""
    ax = grid_axes(n, lo, hi)
    mesh = np.meshgrid(*reversed(ax), indexing="ij")        # slowest axis first
    cols = [m.reshape(-1) for m in reversed(mesh)]           # x, y, (z)
    return np.stack(cols, axis=1)


# -------------------------------------------------------------------------- controls
def controls_2d(m: int) -> np.ndarray:
    """m unit directions at angles 2*pi*k/m.

    When 8 divides m the first octant is evaluated in FP64 and mirrored, so the set
    is exactly invariant under the symmetries of the square (x<->y, sign flips).
    """
    if m % 8 != 0:
        th = 2.0 * math.pi * np.arange(m) / m
        return np.stack([np.cos(th), np.sin(th)], axis=1)
    q4, q8 = m // 4, m // 8
    out = np.empty((m, 2))
    for k in range(m):
        quad, r = divmod(k, q4)
        if r == q8:
            s = math.sqrt(0.5)
            x, y = s, s
        elif r < q8:
            th = 2.0 * math.pi * r / m
            x, y = math.cos(th), math.sin(th)
        else:
            th = 2.0 * math.pi * (q4 - r) / m
            x, y = math.sin(th), math.cos(th)
        for _ in range(quad):            # rotate by +90 degrees per quadrant: exact
            x, y = -y, x
        out[k] = (x + 0.0, y + 0.0)      # + 0.0 turns -0.0 into 0.0
    return out


def controls_3d_fibonacci(m: int) -> np.ndarray:
    """m quasi-uniform unit vectors on the sphere (spherical Fibonacci lattice)."""
    k = np.arange(m, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / m
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def spd_matrix(seed: int, eig=(0.25, 0.5, 1.0)) -> np.ndarray:
    """Q diag(eig) Q^T with Q the sign-fixed QR factor of a seeded 3x3 Gaussian."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))[None, :]
    return q @ np.diag(np.asarray(eig, dtype=np.float64)) @ q.T


# ---------------------------------------------------------------------------- fields
def gaussian_field(shape: Sequence[int], sigma_cells: float, seed: int) -> np.ndarray:
    """White N(0,1) noise FFT-convolved (periodic) with a Gaussian of std sigma_cells,
    then renormalised to mean 0, std 1.  ``shape`` is numpy order (slowest first)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal(tuple(shape))
    spec = np.fft.rfftn(w)
    kern = np.ones(spec.shape)
    for ax, n_ax in enumerate(shape):
        if ax == len(shape) - 1:
            f = np.fft.rfftfreq(n_ax)
        else:
            f = np.fft.fftfreq(n_ax)
        k = np.exp(-2.0 * (math.pi * sigma_cells * f) ** 2)
        sh = [1] * len(shape)
        sh[ax] = k.size
        kern = kern * k.reshape(sh)
    out = np.fft.irfftn(spec * kern, s=tuple(shape), axes=tuple(range(len(shape))))
    out = out - out.mean()
    sd = out.std()
    return out / sd if sd > 0 else out


def f32(a: np.ndarray) -> np.ndarray:
    """Round to float32 and widen back: the stored field is float32-exact."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def separated_centres(k: int, dim: int, sep: float, seed: int, box=0.8,
                      max_tries: int = 100000) -> np.ndarray:
    """k points uniform in [-box, box]^dim with pairwise distance >= sep (rejection)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts: list = []
    tries = 0
    while len(pts) < k:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("cannot place separated centres")
        p = rng.uniform(-box, box, size=dim)
        if all(np.sum((p - q) ** 2) >= sep * sep for q in pts):
            pts.append(p)
    return np.array(pts)


def ball_targets(n, lo, hi, centres: np.ndarray, r: float) -> np.ndarray:
    """int8 target ids: node j belongs to component i iff |x_j - c_i|^2 <= r^2.
    A ball that covers no node gets the node nearest to its centre."""
    X = node_coords(n, lo, hi)
    tid = np.full(X.shape[0], -1, dtype=np.int8)
    for i, c in enumerate(centres):
        d2 = np.sum((X - c[None, :]) ** 2, axis=1)
        inside = d2 <= r * r
        if not inside.any():
            inside = np.zeros_like(inside)
            inside[int(np.argmin(d2))] = True
        tid[inside & (tid < 0)] = i
    return tid


def coarse_stride(n: int, dx: float, r_min: float) -> int:
    """Largest divisor s <= 8 of (n-1) with (n-1)/s >= 16 and s*dx <= r_min, else 1.
    The coarse grid K is then every s-th node of the fine grid."""
    for s in range(8, 1, -1):
        if (n - 1) % s == 0 and (n - 1) // s >= 16 and s * dx <= r_min + 1e-12:
            return s
    return 1


def coarse_nodes_for(n: int, width: float, r_min: float, max_ratio: int = 8,
                     min_nodes: int = 17) -> int:
    """Coarse nodes on an axis of n fine nodes (any count, not nested in general):
    the fewest with a coarse step <= r_min (so every target ball of radius r_min
    holds coarse nodes) and <= max_ratio fine steps, at least min_nodes, at most n."""
    k = max(min_nodes - 1, math.ceil((n - 1) / max_ratio), math.ceil(width / r_min - 1e-9))
    return min(n, k + 1)


# -------------------------------------------------------------------------- problems
def c1_eikonal(n: int = 101, m: int = 32) -> Problem:
    """2D eikonal min-time on [-1,1]^2, f = a (|a| = 1), l = 1, point target at the
    centre node, h = dx.  Closed form of the continuous value: 1 - exp(-|x|)."""
    assert n % 2 == 1
    N = n * n
    tid = np.full(N, -1, dtype=np.int8)
    c = n // 2
    tid[c + n * c] = 0
    return Problem(name=f"eikonal_point_{n}", dim=2, n=(n, n), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                   velocity=controls_2d(m), target=tid, n_comp=1, v_ghost=1.0,
                   coarse_stride=1)


def c2_multitarget(n: int = 1025, m: int = 64, n_disks: int = 4, r: float = 0.05,
                   sigma: float = 0.1, seed_field: int = 102, seed_disks: int = 202) -> Problem:
    """2D, speed c = exp(0.5 g) with g a smoothed unit-variance Gaussian field,
    ``n_disks`` disjoint target disks of radius r."""
    dx = 2.0 / (n - 1)
    g = gaussian_field((n, n), sigma / dx, seed_field)
    c = f32(np.exp(0.5 * g)).reshape(-1)
    cen = separated_centres(n_disks, 2, 0.3, seed_disks)
    tid = ball_targets((n, n), (-1.0, -1.0), (1.0, 1.0), cen, r)
    return Problem(name=f"multitarget_{n}", dim=2, n=(n, n), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                   velocity=controls_2d(m), target=tid, n_comp=n_disks, speed=c, v_ghost=1.0,
                   coarse_stride=coarse_stride(n, dx, r), ra_C=1.0, ra_M=1.0, ra_q=1.0,
                   meta={"centres": cen, "r": r})


def c3_aniso3d(n: int = 257, m: int = 128, n_balls: int = 8, r: float = 0.04,
               sigma: float = 0.1, seed_field: int = 103, seed_balls: int = 203,
               seed_M: int = 303) -> Problem:
    """3D anisotropic: f = c(x) M a with a seeded SPD M (eigenvalues 1/4, 1/2, 1),
    m Fibonacci directions, ``n_balls`` target balls of radius r."""
    dx = 2.0 / (n - 1)
    g = gaussian_field((n, n, n), sigma / dx, seed_field)
    c = f32(np.exp(0.5 * g)).reshape(-1)
    M = spd_matrix(seed_M)
    vel = controls_3d_fibonacci(m) @ M.T
    cen = separated_centres(n_balls, 3, 0.3, seed_balls)
    tid = ball_targets((n, n, n), (-1.0,) * 3, (1.0,) * 3, cen, r)
    return Problem(name=f"aniso3d_{n}", dim=3, n=(n, n, n), lo=(-1.0,) * 3, hi=(1.0,) * 3,
                   velocity=vel, target=tid, n_comp=n_balls, speed=c, v_ghost=1.0,
                   coarse_stride=coarse_stride(n, dx, r), ra_C=1.0, ra_M=1.0, ra_q=1.0,
                   meta={"centres": cen, "r": r, "M": M})


def c4_batch(count: int = 512, seed: int = 404, n_min: int = 16, n_max: int = 512,
             m: int = 32, r: float = 0.05) -> List[Problem]:
    """Independent 2D problems with side lengths log-uniform in [n_min, n_max],
    1-6 target disks each and a smooth seeded speed field (sigma = 0.1 physical).
    The sides are arbitrary, so each coarse grid is chosen by node count
    (``coarse_nodes_for``) rather than by a stride dividing n - 1."""
    out = []
    for p in range(count):
        rng = np.random.Generator(np.random.PCG64(seed + p))
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        k = int(rng.integers(1, 7))
        dx = 2.0 / (n - 1)
        g = gaussian_field((n, n), 0.1 / dx, seed + p + 100000)
        c = f32(np.exp(0.5 * g)).reshape(-1)
        cen = separated_centres(k, 2, 0.3, seed + p + 200000)
        tid = ball_targets((n, n), (-1.0, -1.0), (1.0, 1.0), cen, r)
        nK = coarse_nodes_for(n, 2.0, r)
        out.append(Problem(name=f"batch{p}_{n}", dim=2, n=(n, n), lo=(-1.0, -1.0),
                           hi=(1.0, 1.0), velocity=controls_2d(m), target=tid, n_comp=k,
                           speed=c, v_ghost=1.0, coarse_n=(nK, nK), ra_C=1.0, ra_M=1.0,
                           ra_q=1.0, meta={"centres": cen, "r": r}))
    return out


def c5_adjoint(n: int = 513, m: int = 32, n_disks: int = 4, r: float = 0.05,
               theta_sd: float = 0.1, seed_disks: int = 205, seed_theta: int = 105,
               seed_obs: int = 505, seed_true: int = 605, n_obs: int = 2000,
               swirl: float = 0.0, axis_speed: bool = False) -> Problem:
    """2D learnable-cost problem: f = a, l = exp(theta) with theta i.i.d. N(0, sd^2),
    V_ghost = 2.  ``meta`` holds theta, theta_true and the observation nodes.

    Variants of the same data: ``swirl`` > 0 adds the rotating drift
    swirl * (-x2, x1) (f = drift + a; below 1 the unit controls still steer against
    it everywhere in the box), ``axis_speed`` the per-axis speed factors
    (1 + x1^2 / 2, 1 - x2^2 / 4), so S(x) = diag(c_1, c_2)."""
    N = n * n
    dx = 2.0 / (n - 1)
    cen = separated_centres(n_disks, 2, 0.3, seed_disks)
    tid = ball_targets((n, n), (-1.0, -1.0), (1.0, 1.0), cen, r)
    th = np.random.Generator(np.random.PCG64(seed_theta)).normal(0.0, theta_sd, N)
    th_true = np.random.Generator(np.random.PCG64(seed_true)).normal(0.0, theta_sd, N)
    th = f32(th)
    th_true = f32(th_true)
    obs = obs_nodes(tid, n_obs, seed_obs)
    drift = speed = None
    name = f"adjoint_{n}"
    if swirl > 0.0 or axis_speed:
        X = node_coords((n, n), (-1.0, -1.0), (1.0, 1.0))
        if swirl > 0.0:
            drift = f32(swirl * np.stack([-X[:, 1], X[:, 0]], axis=1))
            name += f"_swirl{swirl}"
        if axis_speed:
            speed = f32(np.stack([1.0 + 0.5 * X[:, 0] ** 2, 1.0 - 0.25 * X[:, 1] ** 2], axis=1))
            name += "_axes"
    return Problem(name=name, dim=2, n=(n, n), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                   velocity=controls_2d(m), target=tid, n_comp=n_disks,
                   cost=f32(np.exp(th)), v_ghost=2.0, drift=drift, speed=speed,
                   coarse_stride=coarse_stride(n, dx, r), ra_C=1.0, ra_M=1.0, ra_q=1.0,
                   meta={"theta": th, "theta_true": th_true, "obs": obs, "centres": cen})


def obs_nodes(target: np.ndarray, k: int, seed: int) -> np.ndarray:
    """k distinct free (non-target) node indices, sorted."""
    free = np.flatnonzero(np.asarray(target) < 0)
    rng = np.random.Generator(np.random.PCG64(seed))
    k = min(k, free.size)
    return np.sort(rng.choice(free, size=k, replace=False)).astype(np.int64)


def strip_problem(n: int, delta: float, m: int = 32) -> Problem:
    """Strip example: targets on the lines x1 = +-1 (split into two components),
    f = a, l = 1, discount lam = delta.  In x2 the grid spans [-1, 1] too; the
    strip's unbounded direction is represented by the ghost value, which is never
    optimal when V_ghost >= 1/delta."""
    N = n * n
    tid = np.full(N, -1, dtype=np.int8)
    T = tid.reshape(n, n)
    T[:, 0] = 1      # x1 = -1
    T[:, -1] = 0     # x1 = +1
    return Problem(name=f"strip_{n}_{delta}", dim=2, n=(n, n), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                   velocity=controls_2d(m), target=tid, n_comp=2, lam=delta,
                   v_ghost=1.0 / delta, coarse_stride=1)


def box_distance_problem(n: int, split: int = 4, m: int = 32) -> Problem:
    """Distance to the boundary of (-1,1)^2 with lam = 1: the whole grid boundary is
    the target, split into ``split`` components (1, 2, 4 edge groups, or 8 half
    edges)."""
    N = n * n
    tid = np.full(N, -1, dtype=np.int8)
    T = tid.reshape(n, n)           # T[i1, i0]
    if split == 1:
        T[0, :] = T[-1, :] = T[:, 0] = T[:, -1] = 0
    elif split == 2:
        T[0, :] = 0; T[:, 0] = 0       # bottom and left
        T[-1, :] = 1; T[:, -1] = 1     # top and right
    elif split == 4:
        T[:, 0] = 3                    # left   (x1 = -1)
        T[-1, :] = 2                   # top    (x2 = +1)
        T[:, -1] = 1                   # right  (x1 = +1)
        T[0, :] = 0                    # bottom (x2 = -1), corners go to the last writer
    elif split == 8:
        h = n // 2                     # each edge in two halves, the middle node to the upper
        T[:h, 0] = 6; T[h:, 0] = 7     # left
        T[-1, :h] = 4; T[-1, h:] = 5   # top
        T[:h, -1] = 2; T[h:, -1] = 3   # right
        T[0, :h] = 0; T[0, h:] = 1     # bottom, corners go to the last writer
    else:
        raise ValueError("split must be 1, 2, 4 or 8")
    return Problem(name=f"boxdist_{n}_{split}", dim=2, n=(n, n), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                   velocity=controls_2d(m), target=tid, n_comp=split, v_ghost=1.0,
                   coarse_stride=1)


def vdp_problem(n: int, split: int = 4, n_a: int = 21, rho: float = 0.2) -> Problem:
    """Van der Pol target problem: f = (x2, (1 - x1^2) x2 - x1) + (0, a), a in [-1,1]
    (``n_a`` values), l = |x|, target = nodes of the ball |x| <= rho split in
    ``split`` slices (halves, quadrants, or octants by angle)."""
    X = node_coords((n, n), (-1.0, -1.0), (1.0, 1.0))
    x1, x2 = X[:, 0], X[:, 1]
    drift = np.stack([x2, (1.0 - x1 * x1) * x2 - x1], axis=1)
    a = np.linspace(-1.0, 1.0, n_a)
    vel = np.stack([np.zeros_like(a), a], axis=1)
    inside = x1 * x1 + x2 * x2 <= rho * rho
    tid = np.full(X.shape[0], -1, dtype=np.int8)
    if split == 1:
        comp = np.zeros(X.shape[0], dtype=np.int8)
    elif split == 2:
        comp = np.where(x2 >= 0, 0, 1).astype(np.int8)
    elif split == 4:
        comp = np.select([(x1 >= 0) & (x2 >= 0), (x1 >= 0) & (x2 < 0), (x1 < 0) & (x2 < 0)],
                         [0, 1, 2], 3).astype(np.int8)
    elif split == 8:
        ang = np.arctan2(x2, x1)                     # (-pi, pi]
        comp = np.clip(np.floor((ang + np.pi) / (np.pi / 4)), 0, 7).astype(np.int8)
    else:
        raise ValueError("split must be 1, 2, 4 or 8")
    tid[inside] = comp[inside]
    return Problem(name=f"vdp_{n}_{split}", dim=2, n=(n, n), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                   velocity=vel, target=tid, n_comp=split, speed=None,
                   cost=f32(np.sqrt(x1 * x1 + x2 * x2)).clip(min=1e-3),
                   drift=f32(drift), v_ghost=2.0, coarse_stride=1)


def circle_controls(m: int, radius: float = 1.0, centre: bool = False) -> np.ndarray:
    """``m`` equally spaced directions of the given length (angle 2 pi k/m, k from
    0), and the zero control appended when ``centre``: a discrete ball for a player
    whose dynamics are linear in its control."""
    th = 2.0 * math.pi * np.arange(m) / m
    v = radius * np.stack([np.cos(th), np.sin(th)], axis=1)
    if centre:
        v = np.vstack([v, np.zeros((1, 2))])
    return v


def pursuit_evasion_problem(n: int, split: int = 4, m_a: int = 32, m_b: int = 8,
                            rho: float = 0.2) -> Problem:
    """Pursuit-evasion game of the paper's Sec. 4.1 on [-1,1]^2: f(x, a, b) =
    (f1(x)(a1 - b1), f2(x)(a2 - b2)) with f1 = x2 + 1, f2 = 1 (per-axis speed
    factors), pursuer a in the unit ball (``m_a`` directions on its circle), evader
    b in the ball of radius 1/2 (``m_b`` directions on its circle and the centre),
    running cost l = x1^2 + 0.1, capture on the ball |x| <= rho split in ``split``
    quadrant-shaped slices."""
    X = node_coords((n, n), (-1.0, -1.0), (1.0, 1.0))
    x1, x2 = X[:, 0], X[:, 1]
    speed = np.stack([x2 + 1.0, np.ones_like(x2)], axis=1)
    inside = x1 * x1 + x2 * x2 <= rho * rho
    tid = np.full(X.shape[0], -1, dtype=np.int8)
    if split == 1:
        comp = np.zeros(X.shape[0], dtype=np.int8)
    elif split == 4:
        comp = np.select([(x1 >= 0) & (x2 >= 0), (x1 >= 0) & (x2 < 0), (x1 < 0) & (x2 < 0)],
                         [0, 1, 2], 3).astype(np.int8)
    else:
        raise ValueError("split must be 1 or 4")
    tid[inside] = comp[inside]
    return Problem(name=f"pe_{n}_{split}", dim=2, n=(n, n), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                   velocity=circle_controls(m_a, 1.0),
                   velocity_b=circle_controls(m_b, 0.5, centre=True),
                   target=tid, n_comp=split, speed=f32(speed), cost=f32(x1 * x1 + 0.1),
                   v_ghost=2.0, coarse_stride=1, ra_C=1.0, ra_M=3.0, ra_q=0.5)


def strip_game_problem(n: int, evader=(-0.5, 0.5), thick: int = 4, n_y: int = 5) -> Problem:
    """A game that moves along x1 only: pursuer a in {-1, +1} e1, evader b in
    ``evader`` (multiples of e1), h = 2 dx, target = the ``thick`` leftmost node
    columns (g = 0).  Feet land on nodes, so the discrete value has a closed form."""
    lo, hi = (-1.0, -1.0), (1.0, 1.0)
    nn = (n, n_y)
    X = node_coords(nn, lo, hi)
    i0 = np.arange(X.shape[0]) % n
    tid = np.where(i0 < thick, 0, -1).astype(np.int8)
    dx = (hi[0] - lo[0]) / (n - 1)
    vel = np.array([[-1.0, 0.0], [1.0, 0.0]])
    vb = np.array([[float(b), 0.0] for b in evader])
    return Problem(name=f"strip_game_{n}", dim=2, n=nn, lo=lo, hi=hi, velocity=vel,
                   velocity_b=vb, target=tid, n_comp=1, h=2.0 * dx, v_ghost=4.0)



def kruzkov_problem(n: int = 513, m: int = 32, n_disks: int = 4, r: float = 0.05,
                    sigma: float = 0.1, seed_field: int = 106, seed_disks: int = 206) -> Problem:
    """Weighted minimum time in its Kruzkov form (``disc = "kruzkov"``): unit speed,
    running cost l = exp(0.5 g) (a slowness field; g a smoothed unit-variance
    Gaussian field), ``n_disks`` capture disks of radius r, v = 1 - exp(-J) with J
    the l-weighted travel time; v_ghost = 2 keeps the initial values a
    supersolution in floating point."""
    dx = 2.0 / (n - 1)
    g = gaussian_field((n, n), sigma / dx, seed_field)
    l = f32(np.exp(0.5 * g)).reshape(-1)
    cen = separated_centres(n_disks, 2, 0.3, seed_disks)
    tid = ball_targets((n, n), (-1.0, -1.0), (1.0, 1.0), cen, r)
    return Problem(name=f"kruzkov_{n}", dim=2, n=(n, n), lo=(-1.0, -1.0), hi=(1.0, 1.0),
                   velocity=controls_2d(m), target=tid, n_comp=n_disks, cost=l, v_ghost=2.0,
                   disc="kruzkov", coarse_stride=coarse_stride(n, dx, r), ra_C=1.0, ra_M=1.0,
                   ra_q=1.0, meta={"centres": cen, "r": r})
