"""Pins of the finite-difference reference (the PDE ground truth).

* w = 1 with identity data: the linear maps are steady solutions of the
  discrete scheme, reproduced to round-off.
* w = 1 sine mode: converges to exp(-2 pi^2 t) phi at second order in h.
* A non-trivial drift: self-convergence at second order (Richardson).
* w = w(x): eta = y exactly (the y-drift vanishes and y is discretely harmonic).
"""
import math

import numpy as np

import workloads as W


def test_linear_maps_are_steady_for_w1(oracle_mod):
    xi, eta = oracle_mod.fd_solve(W.CONST, W.Data(), 0.05, 32, 1e-3)
    x = np.arange(33) / 32
    X, Y = np.meshgrid(x, x)
    assert np.abs(xi - X).max() < 1e-13 and np.abs(eta - Y).max() < 1e-13


def test_sine_mode_second_order(oracle_mod):
    data = W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_SIN)
    t = 0.05
    errs = []
    for n in (16, 32, 64):
        xi, eta = oracle_mod.fd_solve(W.CONST, data, t, n, 1e-4)
        x = np.arange(n + 1) / n
        exact = math.exp(-2 * math.pi ** 2 * t) * np.outer(np.sin(math.pi * x), np.sin(math.pi * x))
        errs.append(np.abs(xi - exact).max())
        assert np.array_equal(xi, eta)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4


def test_bump_self_convergence(oracle_mod):
    dens = W.static_bump()
    vals = []
    for n in (32, 64, 128):
        xi, eta = oracle_mod.fd_solve(dens, W.Data(), 0.02, n, 5e-5)
        step = n // 32
        vals.append(np.stack([xi[::step, ::step], eta[::step, ::step]]))
    d1 = np.abs(vals[1] - vals[0]).max()
    d2 = np.abs(vals[2] - vals[1]).max()
    assert 3.0 < d1 / d2 < 5.0
    # the drift moves the mesh measurably
    assert np.abs(vals[2][0] - np.arange(33)[None, :] / 32).max() > 1e-2


def test_ridge_eta_stays_linear(oracle_mod):
    xi, eta = oracle_mod.fd_solve(W.ridge(), W.Data(), 0.05, 64, 1e-4)
    y = np.arange(65) / 64
    assert np.abs(eta - y[:, None]).max() < 1e-12
    # the problem is symmetric under y -> 1 - y
    assert np.abs(xi - xi[::-1, :]).max() < 1e-12
