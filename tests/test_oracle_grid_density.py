"""Pins of the oracle's grid density: the paper's data path for w, in which w
is known only at grid nodes, grad w comes from finite differences there and
the drift is interpolated bilinearly between the nodes (Sect. 4).

* w = exp(a x) on an n-cell grid: the central difference gives the nodal
  drift -sinh(a h)/h exactly at every interior node, the one-sided
  second-order formulas give -(4 e^{ah} - e^{2ah} - 3)/(2h) at x = 0 and
  -(3 - 4 e^{-ah} + e^{-2ah})/(2h) at x = 1, the y component is 0 to rounding,
  and in between b is linear in x (closed forms at random points; the same
  with x and y exchanged pins the [j][i] orientation).
* The sampled static bump converges to the analytic drift at second order
  in h, and so do the Monte-Carlo estimates on the same paths.
* A sampled ridge w(x) has b_y = 0 (up to rounding), so eta = y in mean.
* Sub-domain solves with the grid density: a ridge keeps eta = y; the
  equidistributed edge data is the cumulative trapezoid sum of the samples
  (w is linear between nodes along an edge).
"""
import math
import os

import numpy as np

import oracle.subdomain as S
import workloads as W

THREADS = min(8, os.cpu_count() or 1)


def nodal(n):
    x = np.arange(n + 1) / n
    return np.meshgrid(x, x)


def exp_grid(n, a, axis):
    X, Y = nodal(n)
    return np.exp(a * (X if axis == 0 else Y))


def exp_nodal_drift(n, a):
    """Closed-form nodal drift of w = exp(a s) along its axis."""
    h = 1.0 / n
    b = np.full(n + 1, -math.sinh(a * h) / h)
    b[0] = -(4 * math.exp(a * h) - math.exp(2 * a * h) - 3) / (2 * h)
    b[n] = -(3 - 4 * math.exp(-a * h) + math.exp(-2 * a * h)) / (2 * h)
    return b


def test_exponential_grid_closed_forms(oracle_mod):
    n, a = 16, 1.3
    rng = np.random.default_rng(5)
    pts = rng.uniform(0, 1, size=(400, 2))
    pts[:8] = [[0, 0], [1, 1], [0.5, 0.25], [1 / 16, 0.3], [15 / 16, 0.7], [0.99, 0.01], [0.01, 0.99], [0.3, 1.0]]
    bn = exp_nodal_drift(n, a)
    for axis in (0, 1):
        dens = W.Density(W.KIND_GRID, w_grid=exp_grid(n, a, axis))
        w, b = oracle_mod.density(dens, 0.0, pts)
        s = pts[:, axis]
        i = np.minimum(np.floor(s * n).astype(int), n - 1)
        f = s * n - i
        expect = (1 - f) * bn[i] + f * bn[i + 1]
        assert np.abs(b[:, axis] - expect).max() < 1e-12 * np.abs(bn).max()
        # zero up to the rounding of the one-sided formula (-3w + 4w - w)
        assert np.abs(b[:, 1 - axis]).max() < 1e-12 * np.abs(bn).max()
        # w between nodes is the bilinear (here: linear) interpolant
        wl = (1 - f) * np.exp(a * i / n) + f * np.exp(a * (i + 1) / n)
        assert np.abs(w - wl).max() < 1e-14 * math.exp(a)


def test_sampled_bump_drift_second_order(oracle_mod):
    dens = W.static_bump()
    pts = W.uniform_points(300, seed=9, lo=0.0, hi=1.0)
    _, exact = oracle_mod.density(dens, 0.0, pts)
    err = []
    for n in (64, 128, 256):
        g = W.Density(W.KIND_GRID, w_grid=oracle_mod.sample_density(dens, 0.0, n))
        _, b = oracle_mod.density(g, 0.0, pts)
        err.append(np.abs(b - exact).max())
    assert err[0] / err[1] > 3.2 and err[1] / err[2] > 3.2, err
    assert err[2] < 0.02 * np.abs(exact).max(), err


def test_sampled_bump_estimates_converge(oracle_mod):
    """Same paths with the sampled and the analytic drift: the estimates
    approach each other at second order in the grid spacing."""
    dens = W.static_bump()
    pts = W.interface_nodes(2, 1, 16)
    t, dt, N = 0.05, 1e-3, 2000
    ref = oracle_mod.fk_solve(dens, W.Data(), pts, t, dt, N, seed=3, threads=THREADS)
    d = []
    for n in (64, 128, 256):
        g = W.Density(W.KIND_GRID, w_grid=oracle_mod.sample_density(dens, 0.0, n))
        o = oracle_mod.fk_solve(g, W.Data(), pts, t, dt, N, seed=3, threads=THREADS)
        d.append(np.abs(o["mean"] - ref["mean"]).max())
    assert d[0] / d[1] > 2.5 and d[1] / d[2] > 2.5, d
    assert d[2] < 0.2 * ref["se"].max(), (d, ref["se"].max())


def test_sampled_ridge_keeps_eta(oracle_mod):
    g = W.Density(W.KIND_GRID, w_grid=oracle_mod.sample_density(W.ridge(), 0.0, 64))
    pts = W.uniform_points(12, seed=2, lo=0.1, hi=0.9)
    _, b = oracle_mod.density(g, 0.0, W.uniform_points(500, seed=4, lo=0.0, hi=1.0))
    assert np.abs(b[:, 1]).max() < 1e-11 and np.abs(b[:, 0]).max() > 1.0
    o = oracle_mod.fk_solve(g, W.Data(), pts, 0.05, 1e-3, 4000, seed=1, threads=THREADS)
    z = (o["mean"][:, 1] - pts[:, 1]) / o["se"][:, 1]
    assert np.abs(z).max() < 4.0, z


def test_subdomain_with_grid_density(oracle_mod):
    N = 24
    X, Y = nodal(N)
    g = W.Density(W.KIND_GRID, w_grid=oracle_mod.sample_density(W.ridge(), 0.0, N))
    xi, eta = S.global_be_step(g, 0.0, 0.05, N, X, Y)
    assert np.abs(eta - Y).max() < 1e-13 and np.abs(xi - X).max() > 1e-3
    # equidistributed edges of a grid density: trapezoid sums of the samples
    ring = W.Density(W.KIND_GRID, w_grid=oracle_mod.sample_density(W.paper_ring(W.TIME_FROZEN, 0.1), 0.1, N))
    gx, gy = S.boundary_grid(N, "equidistributed", ring, 0.0)
    for row, target in ((0, gx[0, :]), (N, gx[N, :])):
        w = ring.w_grid[row, :]
        c = np.concatenate([[0.0], np.cumsum(0.5 * (w[1:] + w[:-1]))])
        assert np.abs(target[1:N] - (c / c[-1])[1:N]).max() < 1e-12
    for col, target in ((0, gy[:, 0]), (N, gy[:, N])):
        w = ring.w_grid[:, col]
        c = np.concatenate([[0.0], np.cumsum(0.5 * (w[1:] + w[:-1]))])
        assert np.abs(target[1:N] - (c / c[-1])[1:N]).max() < 1e-12
