"""Seeded synthetic workloads for the peridynamic hot path.

This module only *generates inputs*: node coordinates and volumes, horizon,
material constants, initial and boundary data, notch geometry and step counts.
It holds none of the method's arithmetic (no neighbour search, no bond law, no
micromodulus calibration, no time stepping), so the GPU path and the CPU
oracle can both be fed from it without sharing any computation.

Node numbering ("original order") is lexicographic with x fastest:
``id = i + nx * (j + ny * k)``.  Every random draw uses
``numpy.random.Generator(PCG64(seed))``.

Geometry follows the EMU nodal discretisation of the paper (Section
"Discretization of peridynamics equations"): one node at the centre of each
cubic/square cell of edge h, nodal volume V = h^d, horizon delta = m h.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

BC_FREE = 0
BC_CLAMPED = 1
BC_VELOCITY = 2


@dataclass
class Workload:
    name: str
    dim: int
    shape: tuple                # nodes per axis
    h: float                    # lattice spacing
    X: np.ndarray               # (n, dim) float64 reference coordinates
    V: np.ndarray               # (n,) float64 nodal volumes
    delta: float                # horizon
    E: float = 1.0              # Young's modulus (calibrates the micromodulus)
    rho: float = 1.0            # mass density
    s_c: float = 0.0            # critical stretch; <= 0 disables damage
    dt: float = 0.0
    steps: int = 0
    u0: Optional[np.ndarray] = None
    v0: Optional[np.ndarray] = None
    bc_kind: Optional[np.ndarray] = None    # (n,) uint8
    bc_vel: Optional[np.ndarray] = None     # (n, dim) float64 prescribed velocity (full value)
    b: Optional[np.ndarray] = None          # (n, dim) body force density or None
    notch: np.ndarray = field(default_factory=lambda: np.zeros((0, 4)))  # (nseg, 4): ax ay bx by
    ramp_steps: int = 0
    fixed: Optional[np.ndarray] = None      # (n,) uint8, implicit problems
    traction: float = 0.0
    precision: str = "fp64"
    seed: Optional[int] = None

    @property
    def n(self) -> int:
        return self.X.shape[0]


def grid_coords(shape, h, jitter=0.0, seed=None):
    """Cell-centred lattice ((i+1/2) h, (j+1/2) h[, (k+1/2) h]), x fastest.

    With ``jitter > 0`` each component is displaced by h * U[-jitter, jitter].
    """
    axes = [(np.arange(s, dtype=np.float64) + 0.5) * h for s in shape]
    mesh = np.meshgrid(*axes, indexing="ij")
    # x fastest: transpose so that flattening in C order runs over axis 0 last
    X = np.stack([m.transpose(tuple(range(len(shape)))[::-1]).reshape(-1) for m in mesh], axis=1)
    if jitter > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        X = X + h * rng.uniform(-jitter, jitter, size=X.shape)
    return np.ascontiguousarray(X)


def lattice_index(shape):
    """Integer lattice coordinates (n, d) in original order."""
    axes = [np.arange(s) for s in shape]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.transpose(tuple(range(len(shape)))[::-1]).reshape(-1) for m in mesh], axis=1)


def plate_2d(N=32, m=3, seed=1, steps=100, modes=4, amplitude=1e-3):
    """Free square plate N x N, h = 1/N, delta = m h, no damage, u0 = 0,
    v0 = seeded sum of sinusoidal modes; dt = 0.1 h.
    """
    h = 1.0 / N
    X = grid_coords((N, N), h)
    n = X.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    v0 = np.zeros((n, 2))
    for _ in range(modes):
        k = rng.integers(1, 5, size=2)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        ang = rng.uniform(0.0, 2.0 * np.pi)
        d = np.array([np.cos(ang), np.sin(ang)])
        v0 += amplitude * np.outer(np.sin(2.0 * np.pi * (X @ k) + phi), d)
    return Workload(
        name=f"plate2d_{N}x{N}_m{m}", dim=2, shape=(N, N), h=h, X=X,
        V=np.full(n, h * h), delta=m * h, E=1.0, rho=1.0, s_c=0.0,
        dt=0.1 * h, steps=steps, u0=np.zeros((n, 2)), v0=v0,
        bc_kind=np.zeros(n, np.uint8), bc_vel=np.zeros((n, 2)), seed=seed)


def notched_plate_2d(N=512, m=4, s_c=1e-3, v0=5e-4, steps=10000, ramp_steps=1000,
                     precision="fp64"):
    """Pre-notched square plate (side L = N h = 1) under opposing edge velocity.

    Notch: horizontal segment at y = floor(N/2) h, x in [0.4 L, 0.6 L].
    Collars: the m bottom rows move with -v0 y-hat, the m top rows with +v0 y-hat,
    ramped linearly over ``ramp_steps`` steps.
    """
    h = 1.0 / N
    L = N * h
    X = grid_coords((N, N), h)
    n = X.shape[0]
    ij = lattice_index((N, N))
    kind = np.zeros(n, np.uint8)
    vel = np.zeros((n, 2))
    bot = ij[:, 1] < m
    top = ij[:, 1] >= N - m
    kind[bot | top] = BC_VELOCITY
    vel[bot, 1] = -v0
    vel[top, 1] = +v0
    yn = (N // 2) * h
    notch = np.array([[0.4 * L, yn, 0.6 * L, yn]])
    return Workload(
        name=f"notched2d_{N}x{N}_m{m}", dim=2, shape=(N, N), h=h, X=X,
        V=np.full(n, h * h), delta=m * h, E=1.0, rho=1.0, s_c=s_c,
        dt=0.1 * h, steps=steps, u0=np.zeros((n, 2)), v0=np.zeros((n, 2)),
        bc_kind=kind, bc_vel=vel, notch=notch, ramp_steps=ramp_steps,
        precision=precision)


def cube_3d(N=100, m=3, jitter=0.05, seed=3, s_c=1e-3, v0=5e-4, steps=2000,
            ramp_steps=200, collar=3, precision="mixed"):
    """Jittered cube N^3, h = 1/N, delta = m h, uniaxial tension along z by
    boundary velocity on ``collar`` planes at each z end (-v0 at the bottom,
    +v0 at the top), ramped over ``ramp_steps`` steps; dt = 0.1 h.
    """
    h = 1.0 / N
    X = grid_coords((N, N, N), h, jitter=jitter, seed=seed)
    n = X.shape[0]
    ijk = lattice_index((N, N, N))
    kind = np.zeros(n, np.uint8)
    vel = np.zeros((n, 3))
    bot = ijk[:, 2] < collar
    top = ijk[:, 2] >= N - collar
    kind[bot | top] = BC_VELOCITY
    vel[bot, 2] = -v0
    vel[top, 2] = +v0
    return Workload(
        name=f"cube3d_{N}^3_m{m}", dim=3, shape=(N, N, N), h=h, X=X,
        V=np.full(n, h ** 3), delta=m * h, E=1.0, rho=1.0, s_c=s_c,
        dt=0.1 * h, steps=steps, u0=np.zeros((n, 3)), v0=np.zeros((n, 3)),
        bc_kind=kind, bc_vel=vel, ramp_steps=ramp_steps, precision=precision,
        seed=seed)


def bar_2d(nx=400, ny=40, m=3, traction=1e-3, clamp_cols=3):
    """Quasi-static bar nx x ny, h = 1/ny (height 1, length nx/ny).

    Columns i < clamp_cols are fixed (u = 0); the last column carries the body
    force density b_x = traction / h, i.e. a traction ``traction`` spread over a
    layer one cell thick.
    """
    h = 1.0 / ny
    X = grid_coords((nx, ny), h)
    n = X.shape[0]
    ij = lattice_index((nx, ny))
    fixed = (ij[:, 0] < clamp_cols).astype(np.uint8)
    b = np.zeros((n, 2))
    b[ij[:, 0] == nx - 1, 0] = traction / h
    return Workload(
        name=f"bar2d_{nx}x{ny}_m{m}", dim=2, shape=(nx, ny), h=h, X=X,
        V=np.full(n, h * h), delta=m * h, E=1.0, rho=1.0, s_c=0.0,
        u0=np.zeros((n, 2)), b=b, fixed=fixed, traction=traction)


# Initial conditions of the paper's 2-d convergence study: a Gaussian pulse
# exp(-|X - x_c|^2 / b) (a1, a2), zero velocity.
CONVERGENCE_ICS = {
    1: {"a": (0.001, 0.0), "xc": (0.5, 0.5), "b": 0.003},
    2: {"a": (0.0002, 0.0007), "xc": (0.25, 0.25), "b": 0.01},
}


def convergence_plate(m, ic, delta=0.1):
    """The 2-d convergence study: material domain [0,1]^2 with the nonlocal
    collar [-delta, 1+delta]^2 - [0,1]^2 clamped (u = 0), h = delta/m on a
    cell-centred grid of the whole square (so meshes with m and 2m nest: each
    coarse cell holds 2 x 2 fine cells), rho = 1, dt = 1e-5, initial
    displacement from CONVERGENCE_ICS[ic] inside [0,1]^2."""
    h = delta / m
    N = int(round((1.0 + 2.0 * delta) / h))
    X = grid_coords((N, N), h) - delta
    n = X.shape[0]
    inside = np.all((X > 0.0) & (X < 1.0), axis=1)
    kind = np.where(inside, BC_FREE, BC_CLAMPED).astype(np.uint8)
    p = CONVERGENCE_ICS[ic]
    g = np.exp(-np.sum((X - np.array(p["xc"])) ** 2, axis=1) / p["b"])
    u0 = np.zeros((n, 2))
    u0[inside] = g[inside, None] * np.array(p["a"])[None, :]
    return Workload(
        name=f"convergence2d_m{m}_ic{ic}", dim=2, shape=(N, N), h=h, X=X,
        V=np.full(n, h * h), delta=delta, E=1.0, rho=1.0, s_c=0.0, dt=1e-5,
        steps=200000, u0=u0, v0=np.zeros((n, 2)), bc_kind=kind, bc_vel=np.zeros((n, 2)))


# initial conditions of the 1-d study: Gaussian pulses a exp(-(x - xc)^2/b)
CONVERGENCE_ICS_1D = {
    1: {"a": 0.001, "xc": (0.5,), "b": 0.003},
    2: {"a": 0.001, "xc": (0.25, 0.75), "b": 0.003},
}
# the 1-d study's influence function J(r) = c1 r exp(-r^2/c2)
INFLUENCE_1D = (1.0, 0.4)


def convergence_line(m, ic, delta=0.01):
    """The 1-d convergence study as a line of nodes in 2-d coordinates
    (y = 0): material domain [0,1] with the nonlocal collar [-delta, 0] and
    [1, 1+delta] clamped (u = 0), h = delta/m on a cell-centred grid of
    [-delta, 1+delta] (meshes with m and 2m nest: each coarse cell holds two
    fine cells), nodal volume h (a length), rho = 1, dt = 1e-5, initial
    displacement (x component) from CONVERGENCE_ICS_1D[ic] inside (0,1)."""
    h = delta / m
    N = int(round((1.0 + 2.0 * delta) / h))
    x = -delta + h * (np.arange(N) + 0.5)
    X = np.stack([x, np.zeros(N)], axis=1)
    inside = (x > 0.0) & (x < 1.0)
    kind = np.where(inside, BC_FREE, BC_CLAMPED).astype(np.uint8)
    p = CONVERGENCE_ICS_1D[ic]
    g = sum(p["a"] * np.exp(-(x - xc) ** 2 / p["b"]) for xc in p["xc"])
    u0 = np.zeros((N, 2))
    u0[inside, 0] = g[inside]
    return Workload(
        name=f"convergence1d_m{m}_ic{ic}", dim=2, shape=(N,), h=h, X=X,
        V=np.full(N, h), delta=delta, E=1.0, rho=1.0, s_c=0.0, dt=1e-5,
        steps=200000, u0=u0, v0=np.zeros((N, 2)), bc_kind=kind, bc_vel=np.zeros((N, 2)))


def coarsen_line(u, N):
    """Average of the two fine cells under each coarse cell (cell-centred
    lines of N and 2N cells)."""
    return 0.5 * (u[0::2] + u[1::2]).reshape(N, -1)


def coarsen(u, N):
    """Average of the 2 x 2 fine cells under each coarse cell (x fastest
    cell-centred grids of N and 2N per side)."""
    f = u.reshape(2 * N, 2 * N, -1)           # [y][x][component]
    return 0.25 * (f[0::2, 0::2] + f[1::2, 0::2] + f[0::2, 1::2] + f[1::2, 1::2]).reshape(N * N, -1)


def random_cloud(n, dim, seed, box=1.0):
    """Uniform random points in [0, box)^dim (for neighbour-search checks)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, box, size=(n, dim))


def dense_cluster(n_cluster, n_side, seed):
    """For delta = 1: n_cluster uniform points in a disk of radius 0.49 about
    the origin (every pair closer than 1, so every row holds n_cluster - 1
    neighbours and the cluster fills one bin), beside an n_side^2 lattice of
    spacing 0.1 at x >= 5 (rows of about 300, bins of about 100)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = 0.49 * np.sqrt(rng.uniform(0.0, 1.0, n_cluster))
    th = 2.0 * np.pi * rng.uniform(0.0, 1.0, n_cluster)
    cl = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    g = grid_coords((n_side, n_side), 0.1) + np.array([5.0, 0.0])
    return np.ascontiguousarray(np.concatenate([cl, g]))


def random_field(n, dim, seed, scale=1e-3):
    rng = np.random.Generator(np.random.PCG64(seed))
    return scale * rng.standard_normal((n, dim))


@dataclass
class Request:
    rid: int
    N: int
    m: int
    s_c: float
    steps: int
    arrival: float


def serving_requests(count=256, seed=5, rate=None, nmin=64, nmax=512):
    """Independent notched-plate requests: side N ~ U{nmin..nmax}, delta in
    {3h, 4h}, s_c ~ U[5e-4, 2e-3], steps ~ U{1000..5000}.  ``rate`` = Poisson
    arrival rate (requests per second); ``None`` means all arrive at t = 0.
    """
    # sizes and arrival gaps from independent streams: the same seed gives
    # the same simulations at any arrival rate
    sz, gap = (np.random.Generator(np.random.PCG64(s))
               for s in np.random.SeedSequence(seed).spawn(2))
    out: List[Request] = []
    t = 0.0
    for r in range(count):
        if rate is not None:
            t += gap.exponential(1.0 / rate)
        out.append(Request(rid=r, N=int(sz.integers(nmin, nmax + 1)),
                           m=int(sz.choice([3, 4])),
                           s_c=float(sz.uniform(5e-4, 2e-3)),
                           steps=int(sz.integers(1000, 5001)), arrival=t))
    return out


def serving_workload(req: "Request") -> Workload:
    """The notched plate of one serving request (edge loading ramped over the
    first fifth of its steps)."""
    return notched_plate_2d(N=req.N, m=req.m, s_c=req.s_c, steps=req.steps,
                            ramp_steps=req.steps // 5, precision="mixed")


CONFIGS = {
    "plate32": lambda: plate_2d(32, 3, seed=1, steps=100),
    # the paper's explicit benchmark shape: 443^2 nodes, horizon of 20 cells
    # (about 1208 neighbours per node), linearised law, no damage
    "paper443": lambda: plate_2d(443, 20, seed=2, steps=100),
    "notched512": lambda: notched_plate_2d(512, 4),
    "cube100": lambda: cube_3d(100, 3),
    "bar400x40": lambda: bar_2d(400, 40, 3),
}
