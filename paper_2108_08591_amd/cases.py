"""Seeded synthetic inputs for the MDF-LBM workloads.

This module produces *inputs only* (case parameters, initial fields, solid
masks); it holds none of the method's arithmetic, and both the GPU path and
the FP64 oracle are driven from it.  Everything is in lattice units
(dx = dt = c = 1, rho0 = 1).

Parameter choices: a case is specified by a target kinematic viscosity nu;
the relaxation rate handed to the solver is the one that yields that nu for
the lattice's cs^2 (the viscosity relation eq. 3-13a solved for s1).  The
Reynolds number of a cavity or channel is Re = U N / nu (Section 4.3).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

# lattice identifiers (same numbering as the C ABI)
D2Q5 = 0
D3Q7 = 1
D2Q4 = 4        # no rest population
D3Q6 = 5        # no rest population
D2Q9 = 8        # diagonal links
D3Q15 = 9       # diagonal links
D2Q9_Q5 = 12    # a lattice per set: velocity sets on D2Q9, the set a = 0 on D2Q5
D3Q15_Q7 = 13   # velocity sets on D3Q15, the set a = 0 on D3Q7
# lattice of the set a = 0 (the lattice itself but for the two ids above)
SET0_LATTICE = {D2Q9_Q5: D2Q5, D3Q15_Q7: D3Q7}
# CS2, NQ and WEIGHTS describe the velocity sets' lattice
CS2 = {D2Q5: 1.0 / 3.0, D3Q7: 1.0 / 4.0, D2Q4: 1.0 / 2.0, D3Q6: 1.0 / 3.0, D2Q9: 1.0 / 3.0, D3Q15: 1.0 / 3.0,
       D2Q9_Q5: 1.0 / 3.0, D3Q15_Q7: 1.0 / 3.0}
DIM = {D2Q5: 2, D3Q7: 3, D2Q4: 2, D3Q6: 3, D2Q9: 2, D3Q15: 3, D2Q9_Q5: 2, D3Q15_Q7: 3}
NQ = {D2Q5: 5, D3Q7: 7, D2Q4: 4, D3Q6: 6, D2Q9: 9, D3Q15: 15, D2Q9_Q5: 9, D3Q15_Q7: 15}
# weights in the population order of the C ABI (eq. d2q5, d3q7, d2q4, d3q6,
# d2q9, d3q15: the printed column order)
WEIGHTS = {D2Q5: [1 / 3] + [1 / 6] * 4, D3Q7: [1 / 4] + [1 / 8] * 6, D2Q4: [1 / 4] * 4, D3Q6: [1 / 6] * 6,
           D2Q9: [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, D3Q15: [2 / 9] + [1 / 9] * 6 + [1 / 72] * 8}
WEIGHTS[D2Q9_Q5] = WEIGHTS[D2Q9]
WEIGHTS[D3Q15_Q7] = WEIGHTS[D3Q15]


def set0_weights(lattice: int) -> list:
    """Weights of the set a = 0 over the q directions of the lattice: those of
    its own lattice, zero-padded where it has fewer directions."""
    w = WEIGHTS[SET0_LATTICE.get(lattice, lattice)]
    return list(w) + [0.0] * (NQ[lattice] - len(w))

PERIODIC = 0
WALL = 1

# forcing schemes (same numbering as the C ABI)
PLAIN = 0        # eq. 3-21: F_i = w_i Fbar added once, ubar = sum_i f
SCHEME2 = 1      # Scheme II, eq. 2-3c / 2-7a


def s1_for_nu(nu: float, lattice: int = D2Q5) -> float:
    """Relaxation rate giving kinematic viscosity nu (eq. 3-13a solved for s1)."""
    return 1.0 / (nu / CS2[lattice] + 0.5)


@dataclasses.dataclass
class CaseSpec:
    """One solver case.  ``shape`` is (nx, ny) or (nx, ny, nz)."""
    lattice: int
    shape: tuple
    s1: float
    s0: float = 1.0
    s2: float = 0.0                      # <= 0: 8(2 - s1)/(8 - s1) (Section 4.1)
    bc: Sequence[int] = (PERIODIC,) * 6  # faces -x,+x,-y,+y,-z,+z
    wall_u: Optional[np.ndarray] = None  # (6, 3)
    force: Sequence[float] = (0.0, 0.0, 0.0)
    R: float = 0.0
    rho0: float = 1.0
    name: str = ""
    forcing: int = PLAIN

    @property
    def d(self) -> int:
        return DIM[self.lattice]

    @property
    def q(self) -> int:
        return NQ[self.lattice]

    @property
    def fshape(self) -> tuple:
        """numpy shape of a scalar field: (ny, nx) or (nz, ny, nx)."""
        return tuple(reversed(self.shape))

    @property
    def nodes(self) -> int:
        return int(np.prod(self.shape))

    def wall_velocity(self) -> np.ndarray:
        return np.zeros((6, 3)) if self.wall_u is None else np.asarray(self.wall_u, float)


# ---------------------------------------------------------------- 2D Taylor-Green

def taylor_green_2d_initial(N: int, u0: float, nu: float):
    """Initial (P, u, grad u) of the decaying 2D Taylor-Green vortex on an
    N x N periodic box, nodes at (i + 1/2, j + 1/2):
      u = -u0 cos(kx) sin(ky), v = u0 sin(kx) cos(ky),
      P = -(u0^2/4)(cos 2kx + cos 2ky),  k = 2 pi / N.
    Returns arrays shaped [y, x] (u, grad component-first)."""
    k = 2.0 * math.pi / N
    x = (np.arange(N) + 0.5)
    X, Y = np.meshgrid(x, x, indexing="xy")
    u = -u0 * np.cos(k * X) * np.sin(k * Y)
    v = u0 * np.sin(k * X) * np.cos(k * Y)
    P = -(u0 * u0 / 4.0) * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    grad = np.empty((2, 2, N, N))
    grad[0, 0] = u0 * k * np.sin(k * X) * np.sin(k * Y)       # du/dx
    grad[0, 1] = -u0 * k * np.cos(k * X) * np.cos(k * Y)      # du/dy
    grad[1, 0] = u0 * k * np.cos(k * X) * np.cos(k * Y)       # dv/dx
    grad[1, 1] = -u0 * k * np.sin(k * X) * np.sin(k * Y)      # dv/dy
    return P, np.stack([u, v]), grad


def tgv2d_case(N: int = 64, u0: float = 0.01, Re: float = 10.0, lattice: int = D2Q5) -> CaseSpec:
    """2D Taylor-Green on a periodic N x N box with Re = u0 N / nu."""
    nu = u0 * N / Re
    return CaseSpec(lattice, (N, N), s1_for_nu(nu, lattice), name=f"tgv2d_{N}")


def tgv2d_convergence_set():
    """Grid-convergence triple: fixed Re and s1, u0 ~ 1/N, steps ~ N^2 (diffusive
    scaling, Remark I).  Returns [(N, u0, nu, steps)]."""
    out = []
    for N, steps in ((32, 250), (64, 1000), (128, 4000)):
        u0 = 0.64 / N
        out.append((N, u0, 0.064, steps))
    return out


# ---------------------------------------------------------------- 3D Taylor-Green

def taylor_green_3d_initial(N: int, u0: float):
    """Initial (P, u) of the 3D Taylor-Green vortex on a periodic N^3 box,
    nodes at (i + 1/2):
      u = u0 sin x cos y cos z, v = -u0 cos x sin y cos z, w = 0,
      P = (u0^2/16)(cos 2x + cos 2y)(cos 2z + 2), with x = k X, k = 2 pi / N.
    Arrays are [z, y, x]."""
    k = 2.0 * math.pi / N
    c = (np.arange(N) + 0.5) * k
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    u = u0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    v = -u0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    w = np.zeros_like(u)
    P = (u0 * u0 / 16.0) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    return P, np.stack([u, v, w])


def tgv3d_case(N: int = 256, u0: float = 0.05, Re: float = 100.0, lattice: int = D3Q7) -> CaseSpec:
    """3D Taylor-Green, Re = u0 N / (2 pi nu) (the usual convention of this
    benchmark: length scale N / 2 pi)."""
    nu = u0 * N / (2.0 * math.pi * Re)
    return CaseSpec(lattice, (N, N, N), s1_for_nu(nu, lattice), name=f"tgv3d_{N}_Re{Re:g}")


# ---------------------------------------------------------------- channel / cavity

def poiseuille_case(nx: int = 256, ny: int = 64, umax: float = 0.05, s1: float = 1.2,
                    lattice: int = D2Q5) -> CaseSpec:
    """Force-driven channel, periodic in x, walls at -y/+y (halfway between
    nodes, so the channel height is H = ny).  Force chosen so that the
    parabolic centreline velocity is umax: F = 8 nu umax / H^2."""
    nu = (1.0 / s1 - 0.5) * CS2[lattice]
    F = 8.0 * nu * umax / (ny * ny)
    return CaseSpec(lattice, (nx, ny), s1, bc=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC),
                    force=(F, 0.0, 0.0), name=f"poiseuille_{nx}x{ny}")


def poiseuille_paper_case() -> CaseSpec:
    """The Poiseuille run of Section 4.1 mapped to lattice units: 32 x 32,
    s1 = 1.2 (nu_lat = 1/9), physical nu = 0.001 on [0, 1] and F1 = 1e-6,
    so dt = nu_lat dx^2 / nu and F_lat = F1 dt^2 / dx."""
    N = 32
    s1 = 1.2
    nu_lat = (1.0 / s1 - 0.5) / 3.0
    dx = 1.0 / N
    dt = nu_lat * dx * dx / 0.001
    F = 1.0e-6 * dt * dt / dx
    return CaseSpec(D2Q5, (N, N), s1, bc=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC),
                    force=(F, 0.0, 0.0), name="poiseuille_paper_32")


def cavity_case(N: int = 1024, Re: float = 1000.0, U: float = 0.1, lattice: int = D2Q5) -> CaseSpec:
    """Lid-driven square cavity, walls on every face, lid = +y face moving
    with (U, 0).  nu = U N / Re."""
    nu = U * N / Re
    wall = np.zeros((6, 3))
    wall[3, 0] = U
    return CaseSpec(lattice, (N, N), s1_for_nu(nu, lattice), bc=(WALL,) * 4 + (PERIODIC, PERIODIC),
                    wall_u=wall, name=f"cavity_{N}_Re{Re:g}")


def couette_case(nx: int = 16, ny: int = 24, U: float = 0.05, s1: float = 1.0,
                 lattice: int = D2Q5) -> CaseSpec:
    """Plane Couette flow: periodic x (and z), resting wall at -y, +y wall
    moving with (U, 0, 0)."""
    wall = np.zeros((6, 3))
    wall[3, 0] = U
    shape = (nx, ny) if DIM[lattice] == 2 else (nx, ny, 4)
    return CaseSpec(lattice, shape, s1, bc=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC),
                    wall_u=wall, name="couette")


def four_roll_mill(N: int = 64, s1: float = 1.2, nu: float = 0.01, U0: float = 1e-4,
                   shift: float = 0.5, lattice: int = D2Q5):
    """The simplified four-roll mill of Section 4.2 on [0, 2 pi]^2 (periodic)
    in lattice units.  Returns (case, force_field[2, y, x], dt, dx): the
    physical force of the section scaled by dt^2/dx with
    dt = nu_lat dx^2 / nu."""
    dx = 2.0 * math.pi / N
    nu_lat = (1.0 / s1 - 0.5) * CS2[lattice]
    dt = nu_lat * dx * dx / nu
    x = (np.arange(N) + shift) * dx
    X, Y = np.meshgrid(x, x, indexing="xy")
    F1 = U0 * U0 * np.sin(X) * np.cos(X) + 2.0 * nu * U0 * np.sin(X) * np.cos(Y)
    F2 = U0 * U0 * np.sin(Y) * np.cos(Y) - 2.0 * nu * U0 * np.sin(Y) * np.cos(X)
    FF = np.stack([F1, F2]) * dt * dt / dx
    return CaseSpec(lattice, (N, N), s1, name=f"fourroll_{N}_s{s1:g}"), FF, dt, dx


# ---------------------------------------------------------------- random states

def random_populations(spec: CaseSpec, seed: int, scale: float = 0.05, rest: float = 1.0):
    """Seeded random pre-collision populations, shape [set][dir] + fshape:
    the rest weights times ``rest`` on the passive set plus uniform noise of
    size ``scale`` everywhere (states far from equilibrium, to exercise every
    term of the collision)."""
    rng = np.random.default_rng(seed)
    q = spec.q
    ns = spec.d + 1
    f = rng.uniform(-scale, scale, size=(ns, q) + spec.fshape)
    w = np.array(set0_weights(spec.lattice))
    f[0] += (rest * w).reshape((q,) + (1,) * spec.d)
    if spec.lattice in SET0_LATTICE:
        f[0, NQ[SET0_LATTICE[spec.lattice]]:] = 0.0      # directions the set a = 0 does not have
    return f


def smooth_random_fields(spec: CaseSpec, seed: int, amp: float = 0.02, modes: int = 3):
    """Seeded smooth periodic velocity and pressure fields (a few random
    Fourier modes), returned as (P, u) with u component-first."""
    rng = np.random.default_rng(seed)
    d = spec.d
    axes = [2 * math.pi * (np.arange(n) + 0.5) / n for n in reversed(spec.shape)]
    grids = np.meshgrid(*axes, indexing="ij")          # [z,]y,x order
    grids = list(reversed(grids))                      # x, y[, z]
    def field():
        acc = np.zeros(spec.fshape)
        for _ in range(modes):
            kv = rng.integers(1, 3, size=d)
            ph = rng.uniform(0, 2 * math.pi)
            arg = sum(kv[b] * grids[b] for b in range(d)) + ph
            acc += rng.uniform(-1, 1) * np.cos(arg)
        return acc
    u = np.stack([amp * field() for _ in range(d)])
    P = amp * amp * field()
    return P, u


# ---------------------------------------------------------------- batched workload

@dataclasses.dataclass
class BatchCase:
    kind: str          # "cavity" or "channel"
    N: int
    Re: float
    U: float
    spec: CaseSpec


def batch_cases(n: int = 512, seed: int = 210808591, nmin: int = 64, nmax: int = 512,
                step: int = 32) -> List[BatchCase]:
    """Uneven batch of independent 2D cavity / channel cases: kind with
    probability 1/2 each, N uniform on {nmin, nmin+step, ..., nmax}, Re
    log-uniform in [10, 1000], U uniform in [0.05, 0.1] (lid speed, or the
    channel centreline speed through F = 8 nu U / N^2); nu = U N / Re."""
    rng = np.random.default_rng(seed)
    sizes = np.arange(nmin, nmax + 1, step)
    out = []
    for _ in range(n):
        kind = "cavity" if rng.random() < 0.5 else "channel"
        N = int(rng.choice(sizes))
        Re = float(10.0 ** rng.uniform(1.0, 3.0))
        U = float(rng.uniform(0.05, 0.1))
        nu = U * N / Re
        s1 = s1_for_nu(nu)
        if kind == "cavity":
            wall = np.zeros((6, 3))
            wall[3, 0] = U
            spec = CaseSpec(D2Q5, (N, N), s1, bc=(WALL,) * 4 + (PERIODIC, PERIODIC), wall_u=wall,
                            name=f"cavity_{N}")
        else:
            F = 8.0 * nu * U / (N * N)
            spec = CaseSpec(D2Q5, (N, N), s1, bc=(PERIODIC, PERIODIC, WALL, WALL, PERIODIC, PERIODIC),
                            force=(F, 0.0, 0.0), name=f"channel_{N}")
        out.append(BatchCase(kind, N, Re, U, spec))
    return out


# ---------------------------------------------------------------- obstacle masks

def obstacle_mask(N: int, rng: np.random.Generator, max_shapes: int = 3, margin: int = 8):
    """Solid mask (uint8, [y, x]) with 0..max_shapes shapes, each a circle
    (radius U(8, 40) nodes) or an axis-aligned rectangle (sides U(16, 80)),
    centres kept at least ``margin`` nodes from every face."""
    mask = np.zeros((N, N), np.uint8)
    ys, xs = np.mgrid[0:N, 0:N] + 0.5
    for _ in range(int(rng.integers(0, max_shapes + 1))):
        cx, cy = rng.uniform(margin, N - margin, size=2)
        if rng.random() < 0.5:
            r = rng.uniform(8, 40) * N / 256.0
            mask[(xs - cx) ** 2 + (ys - cy) ** 2 <= r * r] = 1
        else:
            a, b = rng.uniform(16, 80, size=2) * N / 256.0
            mask[(abs(xs - cx) <= a / 2) & (abs(ys - cy) <= b / 2)] = 1
    # keep a fluid ring next to the walls so every wall node stays fluid
    mask[:2, :] = 0
    mask[-2:, :] = 0
    mask[:, :2] = 0
    mask[:, -2:] = 0
    return mask
