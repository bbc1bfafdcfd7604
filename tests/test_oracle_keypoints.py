"""Pins of the key-point and interpolation oracle (Sect. 4 speed-up, Sect. 5).

* The interpolant equals SciPy's PchipInterpolator (an independent
  implementation of the same Fritsch-Carlson / Fritsch-Butland scheme) on
  random non-uniform knots, reproduces straight lines exactly and keeps
  monotone data monotone.
* Key points of rho(s) = 1 + A exp(-(s - c)^2 / s2) along a line sit at the
  nodes nearest the extrema of rho' (c +- sqrt(s2/2)) and of rho''
  (c and c +- sqrt(3 s2 / 2)), and nowhere else.
* Crossing nodes are always key points; no gap between knots exceeds
  max_gap.
* Interpolating the identity mesh from its key points and boundary ends
  reproduces it at every interface node (canonical-order bookkeeping), and
  a smooth mesh converges at least at second order in the knot spacing.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import PchipInterpolator

import oracle.keypoints as K
import oracle.mesh_step as MS
import oracle.subdomain as S
import workloads as W


@pytest.mark.parametrize("n,seed", [(2, 0), (3, 1), (7, 2), (40, 3)])
def test_pchip_matches_scipy(n, seed):
    rng = np.random.default_rng(seed)
    x = np.sort(rng.uniform(0, 1, n))
    x[0], x[-1] = 0.0, 1.0
    for y in (rng.standard_normal(n), np.cumsum(rng.uniform(0, 1, n)), np.sin(7 * x)):
        q = rng.uniform(0, 1, 500)
        ref = PchipInterpolator(x, y)(q)
        assert np.abs(K.pchip(x, y, q) - ref).max() <= 1e-13 * max(1.0, np.abs(y).max())
        assert np.abs(K.pchip(x, y, x) - y).max() <= 1e-14 * max(1.0, np.abs(y).max())


def test_pchip_lines_and_monotonicity():
    rng = np.random.default_rng(4)
    x = np.sort(rng.uniform(0, 1, 12))
    q = np.linspace(x[0], x[-1], 2001)
    assert np.abs(K.pchip(x, 0.3 - 2.5 * x, q) - (0.3 - 2.5 * q)).max() < 1e-14
    y = np.cumsum(rng.exponential(1.0, 12) * (rng.uniform(size=12) < 0.6))   # with flat stretches
    v = K.pchip(x, y, q)
    assert np.all(np.diff(v) >= -1e-14) and v.min() >= y.min() - 1e-14 and v.max() <= y.max() + 1e-14


def test_keys_at_derivative_extrema():
    N, c, s2, A = 200, 0.37, 0.003, 4.0
    s = np.arange(N + 1) / N
    rho = 1.0 + A * np.exp(-(s - c) ** 2 / s2)
    keys = K.line_keys(rho, m=N, tol=1e-2, max_gap=N)
    targets = [c - math.sqrt(s2 / 2), c + math.sqrt(s2 / 2), c, c - math.sqrt(1.5 * s2), c + math.sqrt(1.5 * s2)]
    assert len(keys) == len(targets), keys
    for t in targets:
        assert min(abs(k / N - t) for k in keys) <= 1.0 / N, (t, keys)
    # through the grid: w = 1/rho(x) -- horizontal lines carry these keys,
    # vertical lines (rho constant along them) only crossings and gap fill
    px, m = 2, 100
    X = np.arange(N + 1) / N
    w = np.tile(1.0 / (1.0 + A * np.exp(-(X - c) ** 2 / s2)), (N + 1, 1))
    mask = K.key_mask(w, px, m, tol=1e-2, max_gap=N)
    ij = S.interface_index(px, m)
    horiz = ij[mask & (ij[:, 1] == m) & (ij[:, 0] != m)][:, 0]
    vert = ij[mask & (ij[:, 0] == m)][:, 1]
    assert sorted(horiz.tolist()) == [k for k in keys if k != m]
    assert vert.tolist() == [m]


@pytest.mark.parametrize("px,m,gap", [(2, 20, 10), (4, 16, 5), (8, 24, 7)])
def test_crossings_and_gaps(oracle_mod, px, m, gap):
    N = px * m
    w = oracle_mod.sample_density(W.paper_ring(W.TIME_FROZEN, 0.3), 0.3, N)
    mask = K.key_mask(w, px, m, tol=1e-2, max_gap=gap)
    ij = S.interface_index(px, m)
    cross = (ij[:, 0] % m == 0) & (ij[:, 1] % m == 0)
    assert np.all(mask[cross])
    for a in range(1, px):
        vertical = ij[mask & (ij[:, 0] == a * m)][:, 1]     # positions along x = a/px
        horizontal = ij[mask & (ij[:, 1] == a * m)][:, 0]   # positions along y = a/px
        for pos in (vertical, horizontal):
            assert np.diff(np.sort(np.concatenate([[0, N], pos]))).max() <= gap
    assert mask.sum() < mask.size            # the speed-up: fewer simulated nodes


def test_identity_mesh_reproduced(oracle_mod):
    px, m = 4, 16
    N = px * m
    w = oracle_mod.sample_density(W.two_bumps(W.TIME_FROZEN, 0.02), 0.02, N)
    mask = K.key_mask(w, px, m, tol=1e-2, max_gap=6)
    pts = MS.interface_points(px, m)
    X, Y = np.meshgrid(np.arange(N + 1) / N, np.arange(N + 1) / N)
    out = K.interpolate_interface(px, m, mask, pts[mask], X, Y)
    assert np.abs(out - pts).max() < 1e-14


def test_smooth_mesh_converges():
    px, m = 2, 64
    N = px * m
    X, Y = np.meshgrid(np.arange(N + 1) / N, np.arange(N + 1) / N)
    f = (X + 0.05 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y), Y + 0.04 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y))
    pts = MS.interface_points(px, m)
    exact = np.stack([f[c][np.rint(pts[:, 1] * N).astype(int), np.rint(pts[:, 0] * N).astype(int)] for c in (0, 1)], 1)
    err = []
    for gap in (16, 8, 4):
        mask = K.key_mask(np.ones((N + 1, N + 1)), px, m, max_gap=gap)
        out = K.interpolate_interface(px, m, mask, exact[mask], f[0], f[1])
        err.append(np.abs(out - exact).max())
    assert err[0] / err[1] > 3.5 and err[1] / err[2] > 3.5, err


def test_keyed_step_w1_identity(oracle_mod):
    """w = 1 from the identity mesh: the key-point step keeps the identity
    within the Monte-Carlo error of its key estimates."""
    px, m, D = 2, 20, 1e-3
    N = px * m
    X, Y = np.meshgrid(np.arange(N + 1) / N, np.arange(N + 1) / N)
    w = np.ones((N + 1, N + 1))
    xi, eta, mc, mask = MS.dd_step_keys(W.CONST, 0.0, D, 20, px, m, X, Y, 4000, w, max_gap=5, threads=4)
    assert 0 < mask.sum() < mask.size
    tol = 4.5 * mc["se"].max()
    assert np.abs(xi - X).max() <= tol and np.abs(eta - Y).max() <= tol
