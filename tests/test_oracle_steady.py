"""Pins of the elliptic (steady) variant: the system of eq. (2),
grad . ((1/w) grad xi) = 0, i.e. Laplacian xi - (grad w / w) . grad xi = 0,
with its Feynman-Kac representation xi(P) = E[g(X_tau)] (paths run until
they leave the square).

* Steady solves: w = 1 keeps the linear maps; w = w(x) with the
  equidistributed boundary data keeps eta = y and gives
  xi = int_0^x w / int_0^1 w (the 1-D equidistribution, exact for the PDE)
  at second order in h; the steady rows are the limit of the
  backward-Euler ones (D = 1e9 agrees to ~1e-8); with the global steady
  solution's interface values the sub-domain solves reproduce it (exact DD
  identity).
* Monte Carlo: for w = w(x) with the same boundary data the estimates of xi
  follow the closed form within their error, and eta = y.
"""
import math
import os

import numpy as np
import pytest
import scipy.integrate as si

import oracle.mesh_step as MS
import oracle.subdomain as S
import workloads as W

THREADS = min(8, os.cpu_count() or 1)


def nodal(N):
    x = np.arange(N + 1) / N
    return np.meshgrid(x, x)


def equidistribution(dens, x):
    w = lambda s: 1.0 + dens.amp * math.exp(-(s - dens.cx) ** 2 / dens.width2)  # noqa: E731
    total = si.quad(w, 0, 1, epsabs=1e-14)[0]
    return np.array([si.quad(w, 0, v, epsabs=1e-14)[0] / total for v in np.atleast_1d(x)])


def test_steady_w1_linear_maps():
    X, Y = nodal(20)
    xi, eta = S.global_be_step(W.CONST, 0.0, np.inf, 20, None, None)
    assert np.abs(xi - X).max() < 1e-13 and np.abs(eta - Y).max() < 1e-13


def test_steady_ridge_closed_form_second_order():
    dens = W.ridge()
    err = []
    for N in (16, 32, 64):
        X, Y = nodal(N)
        xi, eta = S.global_be_step(dens, 0.0, np.inf, N, None, None, bdry="equidistributed")
        assert np.abs(eta - Y).max() < 1e-12
        exact = equidistribution(dens, X[0])
        err.append(np.abs(xi - exact[None, :]).max())
    assert err[0] / err[1] > 3.5 and err[1] / err[2] > 3.5, err


def test_steady_is_the_limit_of_backward_euler():
    N = 24
    X, Y = nodal(N)
    dens = W.static_bump()
    a = S.global_be_step(dens, 0.0, np.inf, N, None, None)
    b = S.global_be_step(dens, 0.0, 1e9, N, X, Y)
    assert max(np.abs(a[0] - b[0]).max(), np.abs(a[1] - b[1]).max()) < 1e-7
    assert np.abs(a[0] - X).max() > 1e-3


@pytest.mark.parametrize("px,m,dens,bdry", [(4, 8, W.static_bump(), "identity"),
                                            (2, 20, W.paper_ring(W.TIME_FROZEN, 0.0), "equidistributed")])
def test_steady_exact_domain_decomposition(px, m, dens, bdry):
    N = px * m
    gx, gy = S.global_be_step(dens, 0.0, np.inf, N, None, None, bdry=bdry)
    ij = S.interface_index(px, m)
    sx, sy = S.subdomain_be_step(dens, 0.0, np.inf, px, m, None, None, gx[ij[:, 1], ij[:, 0]],
                                 gy[ij[:, 1], ij[:, 0]], bdry=bdry)
    assert max(np.abs(sx - gx).max(), np.abs(sy - gy).max()) < 1e-12


def test_elliptic_monte_carlo_ridge(oracle_mod):
    dens = W.ridge()
    pts = np.array([[0.2, 0.5], [0.3, 0.25], [0.35, 0.7], [0.45, 0.5], [0.6, 0.4], [0.8, 0.6]])
    sx, sy = MS.steady_start(2, 32, "equidistributed", dens)
    data = W.Data(init_kind=W.DATA_GRID, bdry_kind=W.DATA_GRID, score_mode=W.SCORE_BRIDGE, grid_xi=sx, grid_eta=sy)
    o = oracle_mod.fk_solve(dens, data, pts, 3.0, 1e-4, 4000, seed=7, want_exit=True, threads=THREADS)
    assert np.all(o["exit_step"] > 0)                        # every path left the square
    z_eta = (o["mean"][:, 1] - pts[:, 1]) / o["se"][:, 1]
    assert np.all(np.abs(z_eta) < 4.5), z_eta
    d = o["mean"][:, 0] - equidistribution(dens, pts[:, 0])
    assert np.all(np.abs(d) < 4.5 * o["se"][:, 0] + 1e-3), (d, o["se"][:, 0])
