"""Seeded synthetic inputs for the stochastic interface solver.

This module is shared by the CPU oracle tests, the GPU parity tests and the
benchmark.  It holds parameter sets and node placements only: nothing in here
evaluates a density, a drift, a path or an estimator, so it carries none of the
method's arithmetic.

Workloads (all synthetic; the paper's experiment uses an analytic density too,
Sect. 5):

* ``static_bump``     -- w = 1 + 10 exp(-|X-(0.3,0.6)|^2/0.01), two sub-domains
                         split at x = 1/2, 31 interface nodes, t = 0.05, dt = 1e-4.
* ``moving_bump``     -- w = 1 + 20 exp(-|X-c(tau)|^2/0.005) with the bump centre
                         c(tau) = (1/2 + cos(2 pi tau)/4, 1/2 + sin(2 pi tau)/4)
                         following the paper's moving centre (Sect. 5); 4x4
                         sub-domains, 255 nodes per interface line, 1521 unique
                         nodes, t = 0.1, dt = 1e-5.
* ``two_bumps``       -- two counter-rotating bumps (amplitude 30, width^2 0.003)
                         for the time-dependent mesh run.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

# Density kinds (w(tau, x, y)).
KIND_CONST = 0        # w = 1
KIND_BUMP = 1         # w = 1 + A exp(-|X - (cx, cy)|^2 / s2)
KIND_MOVING_BUMP = 2  # centre (cx + R cos(omega tau), cy + R sin(omega tau))
KIND_TWO_BUMPS = 3    # second centre mirrored in x: (cx - R cos(omega tau), cy + R sin(omega tau))
KIND_RING = 4         # the paper's w = 1/rho moving ring (Sect. 5); amp = alpha, width2 = beta
KIND_RIDGE = 5        # w = 1 + A exp(-(x - cx)^2 / s2): depends on x only
KIND_GRID = 6         # w known at the nodes of a grid only (Sect. 4): samples in Density.w_grid

# Which time argument the density takes along a path.
TIME_BACKWARD = 0     # w(t_init + t - s): the Feynman-Kac time reversal
TIME_FROZEN = 1       # w(t_freeze): held fixed over one mesh step (Sect. 4)

# Initial / boundary data kinds.
DATA_IDENTITY = 0     # xi = x, eta = y (initial uniform mesh, Sect. 3)
DATA_SIN = 1          # both components phi = sin(pi x) sin(pi y); boundary data the
                      # decaying mode exp(-2 pi^2 s') phi extended off the square
DATA_ZERO = 2         # boundary data 0
DATA_GRID = 3         # initial data bilinear in a (n+1)^2 nodal grid (initial data only)
DATA_EQUIDISTRIBUTED = 4  # outer boundary of the sub-domain solves: 1-D equidistribution on two edges

SCORE_UNCLAMPED = 0   # evaluate the boundary data at the (unclamped) first outside point
SCORE_PROJECT = 1     # clamp that point onto the closed square first
SCORE_EXTEND = 2      # the grid initial data continued bilinearly to that point
SCORE_BRIDGE = 3      # Brownian-bridge exit test within each step; exits scored at the projected point
SCORE_EXPONENTIAL = 4  # exponentially distributed step lengths (mean dt) with the bridge test; exits projected

# Philox stream tags (low 4 bits of the last counter word).
STREAM_PATHS = 0
STREAM_LABELS = 1
STREAM_MINIBATCH = 2
STREAM_MLP_INIT = 3


@dataclass(frozen=True)
class Density:
    kind: int
    time_mode: int = TIME_BACKWARD
    amp: float = 0.0
    width2: float = 1.0
    cx: float = 0.5
    cy: float = 0.5
    orbit_r: float = 0.0
    omega: float = 0.0
    t_freeze: float = 0.0
    w_grid: np.ndarray | None = field(default=None, compare=False)   # KIND_GRID: [(n+1), (n+1)] [j, i]

    @property
    def w_n(self) -> int:
        return 0 if self.w_grid is None else int(self.w_grid.shape[0]) - 1

    def params(self) -> np.ndarray:
        """The 7 real parameters in the order both implementations read them."""
        return np.array([self.amp, self.width2, self.cx, self.cy, self.orbit_r,
                         self.omega, self.t_freeze], dtype=np.float64)


@dataclass(frozen=True)
class Data:
    init_kind: int = DATA_IDENTITY
    bdry_kind: int = DATA_IDENTITY
    score_mode: int = SCORE_UNCLAMPED
    t_init: float = 0.0
    grid_xi: np.ndarray | None = field(default=None, compare=False)
    grid_eta: np.ndarray | None = field(default=None, compare=False)

    @property
    def grid_n(self) -> int:
        return 0 if self.grid_xi is None else int(round(math.sqrt(self.grid_xi.size))) - 1


CONST = Density(KIND_CONST)


def static_bump() -> Density:
    return Density(KIND_BUMP, TIME_BACKWARD, amp=10.0, width2=0.01, cx=0.3, cy=0.6)


def moving_bump(time_mode: int = TIME_BACKWARD, t_freeze: float = 0.0) -> Density:
    return Density(KIND_MOVING_BUMP, time_mode, amp=20.0, width2=0.005, cx=0.5, cy=0.5,
                   orbit_r=0.25, omega=2.0 * math.pi, t_freeze=t_freeze)


def two_bumps(time_mode: int = TIME_FROZEN, t_freeze: float = 0.0) -> Density:
    return Density(KIND_TWO_BUMPS, time_mode, amp=30.0, width2=0.003, cx=0.5, cy=0.5,
                   orbit_r=0.25, omega=2.0 * math.pi, t_freeze=t_freeze)


def ridge(amp: float = 10.0, width2: float = 0.01, cx: float = 0.35) -> Density:
    return Density(KIND_RIDGE, TIME_BACKWARD, amp=amp, width2=width2, cx=cx)


def paper_ring(time_mode: int = TIME_FROZEN, t_freeze: float = 0.0) -> Density:
    """w = 1/rho with rho = 1 + alpha exp(beta |r^2 - 1/100|), alpha = 10, beta = -50 (Sect. 5)."""
    return Density(KIND_RING, time_mode, amp=10.0, width2=-50.0, cx=0.5, cy=0.5,
                   orbit_r=0.25, omega=2.0 * math.pi, t_freeze=t_freeze)


def interface_nodes(px: int, py: int, G: int) -> np.ndarray:
    """Interface nodes of a px x py sub-domain layout of the unit square.

    Canonical order: the vertical lines x = i/px (i = 1..px-1, ascending), each
    with nodes y = j/G (j = 1..G-1, ascending); then the horizontal lines
    y = k/py with nodes x = j/G, skipping nodes already listed (crossings).
    Nodes on the outer boundary are never included.  A horizontal-line node
    (j/G, k/py) is a duplicate exactly when it lies on a vertical line
    (j px divisible by G) at one of that line's nodes (k G divisible by py).
    """
    pts = []
    for i in range(1, px):
        for j in range(1, G):
            pts.append((i / px, j / G))
    for k in range(1, py):
        on_node_row = (k * G) % py == 0
        for j in range(1, G):
            if on_node_row and (j * px) % G == 0:
                continue
            pts.append((j / G, k / py))
    return np.array(pts, dtype=np.float64).reshape(-1, 2)


@dataclass(frozen=True)
class Workload:
    name: str
    density: Density
    px: int
    py: int
    G: int
    t: float
    dt: float
    n_paths: int
    seed: int = 0
    data: Data = Data()

    def nodes(self) -> np.ndarray:
        return interface_nodes(self.px, self.py, self.G)

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# Plain MC, FP64-CPU-sized case: 2 sub-domains split at x = 1/2, 31 nodes.
STATIC_BUMP_31 = Workload("static_bump_31", static_bump(), px=2, py=1, G=32,
                          t=0.05, dt=1e-4, n_paths=10_000)

# Plain MC on the moving bump: 4x4 sub-domains, 1521 unique interface nodes.
MOVING_BUMP_1521 = Workload("moving_bump_1521", moving_bump(), px=4, py=4, G=256,
                            t=0.1, dt=1e-5, n_paths=100_000)


def random_layouts(n_levels: int = 64, lo: int = 2, hi: int = 8, seed: int = 0):
    """Sub-domain layouts (px, py) drawn uniformly from {lo..hi}^2, one per time level."""
    rng = np.random.default_rng(seed)
    return [(int(a), int(b)) for a, b in rng.integers(lo, hi + 1, size=(n_levels, 2))]


def batched_levels(n_levels: int = 64, G: int = 128, dt_level: float = 0.01, seed: int = 0):
    """Time levels t_k = k * dt_level (k = 1..n_levels), each with a random layout.

    Returns a list of (t_k, px, py, nodes[n_k, 2]).
    """
    out = []
    for k, (px, py) in enumerate(random_layouts(n_levels, seed=seed), start=1):
        out.append((k * dt_level, px, py, interface_nodes(px, py, G)))
    return out


def uniform_points(n: int, seed: int, lo: float = 0.02, hi: float = 0.98) -> np.ndarray:
    """n seeded uniform points inside the unit square (parity tests)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(n, 2))


# ---------------------------------------------------------------------------
# Control-variate network inputs: initial weights and the training set.
# ---------------------------------------------------------------------------
MLP_SHAPES = [(64, 3), (64,), (64, 64), (64,), (64, 64), (64,), (2, 64), (2,)]
MLP_N_PARAMS = 8706
CV_T_SCALE = 0.1     # network time input z0 = 2 t / T - 1 over [0, T]


def mlp_init(seed: int = 0) -> np.ndarray:
    """Flat initial parameters: Glorot-uniform weights, zero biases (FP32 values)."""
    rng = np.random.default_rng(seed)
    out = []
    for shape in MLP_SHAPES:
        if len(shape) == 2:
            a = math.sqrt(6.0 / (shape[0] + shape[1]))
            out.append(rng.uniform(-a, a, size=shape).astype(np.float32).ravel())
        else:
            out.append(np.zeros(shape, dtype=np.float32))
    flat = np.concatenate(out)
    assert flat.size == MLP_N_PARAMS
    return flat


def cv_label_levels(n_levels: int = 132, t_max: float = 0.1):
    """Time levels t_m = t_max m / (n_levels - 1), m = 0..n_levels-1, of the training labels."""
    return [t_max * m / (n_levels - 1) for m in range(n_levels)]
