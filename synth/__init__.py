"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds problem descriptions (plain data) and the seeded random
inputs: base flows q0, start vectors, right-hand sides and per-problem
parameter draws.  It contains none of the stability method's arithmetic
(no derivatives, no operator, no solver); both the CPU oracle and the HIP
path receive what it produces as plain arrays.

Problem setup follows the model problem of the paper (Section "Model
problem", eq. tanh): a temporal mixing layer with u1 = u_inf tanh(x2/delta),
non-dimensionalised with u_inf = delta = rho_ref = T_ref = 1.  The domain is
periodic in x (and z in 3D) and bounded by walls at y = +-Ly/2; the wall rows
belong to the grid (Ny counts them) and every perturbation vanishes there.

Vector layout (struct of arrays, x fastest):
    2D: q[var, j, i]      var in (p, u, v, s)
    3D: q[var, k, j, i]   var in (p, u, v, w, s)
flattened C-order, so idx = ((var*Nz + k)*Ny + j)*Nx + i.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

GAMMA = 1.4
PRANDTL = 0.72
# Sutherland temperature over the reference temperature (110.4 K / 288.15 K).
SUTHERLAND = 110.4 / 288.15

BC_PERIODIC = 0
BC_WALL = 1

# first-derivative schemes of the discrete operator
SCHEME_EXPLICIT = 0   # explicit 6th-order central differences
SCHEME_COMPACT = 1    # 6th-order compact (tridiagonal) differences


@dataclass(frozen=True)
class Problem:
    """Plain description of one base-flow problem (no derived arithmetic)."""
    ndim: int                       # 2 or 3
    n: Tuple[int, int, int]         # (Nx, Ny, Nz); Nz = 1 in 2D; Ny includes both walls
    length: Tuple[float, float, float]  # (Lx, Ly, Lz); y spans [-Ly/2, Ly/2]
    mach: float
    re: float                       # re <= 0 means inviscid
    pr: float = PRANDTL
    gamma: float = GAMMA
    sutherland: float = SUTHERLAND
    bc: Tuple[int, int, int] = (BC_PERIODIC, BC_WALL, BC_PERIODIC)
    scheme: int = SCHEME_EXPLICIT
    stretch: float = 0.0            # y-grid stretching beta (0: uniform; walls in y only)

    @property
    def nv(self) -> int:
        return 4 if self.ndim == 2 else 5

    @property
    def npts(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def ndof(self) -> int:
        return self.nv * self.npts

    @property
    def shape(self) -> Tuple[int, ...]:
        nx, ny, nz = self.n
        if self.ndim == 2:
            return (self.nv, ny, nx)
        return (self.nv, nz, ny, nx)


LX_MIXING = 2.0 * math.pi / 0.4     # one wavelength of alpha = 0.4
LY_MIXING = 30.0                    # y in [-15, 15]


def mixing_layer_2d(nx: int, ny: int, mach: float, re: float,
                    lx: float = LX_MIXING, ly: float = LY_MIXING,
                    bc_y: int = BC_WALL, scheme: int = SCHEME_EXPLICIT, stretch: float = 0.0) -> Problem:
    return Problem(ndim=2, n=(nx, ny, 1), length=(lx, ly, 1.0), mach=mach, re=re,
                   bc=(BC_PERIODIC, bc_y, BC_PERIODIC), scheme=scheme, stretch=stretch)


def mixing_layer_3d(nx: int, ny: int, nz: int, mach: float, re: float,
                    lx: float = LX_MIXING, ly: float = LY_MIXING,
                    lz: float | None = None, bc_y: int = BC_WALL,
                    scheme: int = SCHEME_EXPLICIT, stretch: float = 0.0) -> Problem:
    if lz is None:
        lz = lx / 2.0
    return Problem(ndim=3, n=(nx, ny, nz), length=(lx, ly, lz), mach=mach, re=re,
                   bc=(BC_PERIODIC, bc_y, BC_PERIODIC), scheme=scheme, stretch=stretch)


# ---------------------------------------------------------------------------
# The five benchmark workloads (Cayley shifts sigma, mu and the Arnoldi sizes
# are the same in all of them).
# ---------------------------------------------------------------------------
SIGMA = 0.2
MU = -0.2
NCV = 30
NEV = 6


def config0() -> Problem:
    """2D mixing layer 48x48, M=0.3, Re=500 (full eigen parity case)."""
    return mixing_layer_2d(48, 48, 0.3, 500.0)


def config1() -> Problem:
    """2D mixing layer 512x512, M=0.5, Re=1000 (Jv throughput, GMRES(40))."""
    return mixing_layer_2d(512, 512, 0.5, 1000.0)


def config2() -> Problem:
    """3D mixing layer 256x128x128 (x, z periodic), M=0.5, Re=1000."""
    return mixing_layer_3d(256, 128, 128, 0.5, 1000.0)


def config3_shifts() -> List[float]:
    """Eight evenly spaced Cayley shifts 0.05 .. 0.40 for the block-Jacobi case."""
    return [0.05 * (k + 1) for k in range(8)]


@dataclass(frozen=True)
class SweepItem:
    problem: Problem
    seed: int


def config4_sweep(seed: int = 4, count: int = 48) -> List[SweepItem]:
    """48 uneven 2D base flows: side uniform on {128, 144, ..., 768},
    M ~ U[0.1, 0.8], Re ~ U[300, 2000], all drawn from the seed."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(4)[3])
    sides = np.arange(128, 769, 16)
    out = []
    for i in range(count):
        side = int(rng.choice(sides))
        mach = float(rng.uniform(0.1, 0.8))
        re = float(rng.uniform(300.0, 2000.0))
        out.append(SweepItem(mixing_layer_2d(side, side, mach, re), seed * 1000 + i))
    return out


def config4_reduced(seed: int = 4, count: int = 8, sides=(24, 32, 40, 48)) -> List[SweepItem]:
    """The sweep's recipe (M ~ U[0.1, 0.8], Re ~ U[300, 2000], side drawn
    uniformly, all from the seed) on small sides, so that every problem's
    Cayley-IRAM finishes in seconds with unpreconditioned inner solves."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(4)[3])
    sides = np.asarray(sides)
    out = []
    for i in range(count):
        side = int(rng.choice(sides))
        mach = float(rng.uniform(0.1, 0.8))
        re = float(rng.uniform(300.0, 2000.0))
        out.append(SweepItem(mixing_layer_2d(side, side, mach, re), seed * 1000 + i))
    return out


# ---------------------------------------------------------------------------
# Grids and base flows.
# ---------------------------------------------------------------------------
def grid_y(prob: Problem) -> np.ndarray:
    """y coordinates: Ny points including both walls; uniform, or with
    stretch = beta > 0 the points y = (Ly/2) sinh(beta eta) / sinh(beta) of a
    uniform eta grid on [-1, 1] (clustered around the layer's centre y = 0,
    as the paper's grid is around the largest velocity gradients)."""
    ny = prob.n[1]
    ly = prob.length[1]
    if prob.stretch > 0.0:
        eta = -1.0 + np.arange(ny) * (2.0 / (ny - 1))
        return 0.5 * ly * np.sinh(prob.stretch * eta) / np.sinh(prob.stretch)
    return -0.5 * ly + np.arange(ny) * (ly / (ny - 1))


def base_pressure(prob: Problem) -> float:
    """Uniform base pressure p = 1/(gamma M^2) for rho = T = 1."""
    return 1.0 / (prob.gamma * prob.mach ** 2)


def wall_mask(prob: Problem) -> np.ndarray:
    """Boolean array of the field shape (without the var axis): True on wall rows."""
    nx, ny, nz = prob.n
    m = np.zeros((ny, nx), dtype=bool)
    if prob.bc[1] == BC_WALL:
        m[0, :] = True
        m[-1, :] = True
    if prob.ndim == 3:
        m = np.broadcast_to(m, (nz, ny, nx)).copy()
    return m


def _streams(seed: int):
    return np.random.SeedSequence(seed).spawn(4)


def base_flow(prob: Problem, seed: int = 0, w_noise: float = 0.0) -> np.ndarray:
    """tanh mixing layer: u = tanh(y), v = 0, uniform p and T (s = 0).

    In 3D, w = w_noise * N(0,1) per point (0 on the walls), drawn from the
    seed's base-noise stream.  Returns float64 of shape prob.shape."""
    q = np.zeros(prob.shape, dtype=np.float64)
    y = grid_y(prob)
    q[0] = base_pressure(prob)
    if prob.ndim == 2:
        q[1] = np.tanh(y)[:, None]
    else:
        q[1] = np.tanh(y)[None, :, None]
        if w_noise != 0.0:
            rng = np.random.default_rng(_streams(seed)[2])
            w = w_noise * rng.standard_normal(prob.shape[1:])
            w[wall_mask(prob)] = 0.0
            q[3] = w
    return q


def random_vector(prob: Problem, seed: int, stream: int = 0, scale: float = 1.0,
                  nrhs: int = 1) -> np.ndarray:
    """Seeded N(0,1) vector(s) in the interior subspace (wall entries 0).

    stream 0: start vectors, 1: right-hand sides.  Shape (nrhs, *prob.shape)
    if nrhs > 1 else prob.shape."""
    rng = np.random.default_rng(_streams(seed)[stream])
    out = scale * rng.standard_normal((nrhs,) + prob.shape)
    m = wall_mask(prob)
    for r in range(nrhs):
        for var in range(prob.nv):
            out[r, var][m] = 0.0
    return out if nrhs > 1 else out[0]


def random_base(prob: Problem, seed: int, amp: float = 0.05) -> np.ndarray:
    """A generic smooth-ish, non-uniform base state for operator tests: the
    tanh layer plus seeded perturbations of every variable (p and s included,
    so that every base-derivative term of the operator is exercised)."""
    rng = np.random.default_rng(_streams(seed)[3])
    q = base_flow(prob)
    q = q + amp * rng.standard_normal(q.shape)
    q[0] = base_pressure(prob) * (1.0 + amp * rng.standard_normal(q.shape[1:]))
    return q
