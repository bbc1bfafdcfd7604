"""Pins of the control-variate (Dynkin-form) oracle.

* u_hat = 0 reproduces the plain estimate bit for bit.
* w = 1 with the exact solution as u_hat (identity data and u_hat = (x, y);
  the sine mode and u_hat its exact decaying solution): every path scores
  the same number, so the estimate is exact with zero variance, for any dt
  and any stride.
* A linear u_hat with w != 1: the telescoping sum is exact in expectation,
  so the CV estimate agrees with the plain one within their standard errors
  (and the CV variance is lower where the drift is strong).
* A trained-looking network: CV and plain agree within 3 combined standard
  errors on the same paths.
"""
import math

import numpy as np

import oracle.mlp as M
import workloads as W


def test_zero_uhat_is_plain(oracle_mod):
    pts = W.uniform_points(6, seed=1)
    cv = oracle_mod.fk_solve_cv(W.static_bump(), W.Data(), pts, 0.02, 1e-4, 500, seed=3, uhat=oracle_mod.UHAT_ZERO)
    pl = oracle_mod.fk_solve(W.static_bump(), W.Data(), pts, 0.02, 1e-4, 500, seed=3)
    assert np.array_equal(cv["mean"], pl["mean"]) and np.array_equal(cv["se"], pl["se"])
    assert np.array_equal(cv["plain_mean"], pl["mean"])


def test_exact_uhat_gives_zero_variance(oracle_mod):
    pts = W.uniform_points(8, seed=2)
    for stride in (1, 3):
        r = oracle_mod.fk_solve_cv(W.CONST, W.Data(), pts, 0.05, 2e-3, 400, seed=1,
                                   uhat=oracle_mod.UHAT_LINEAR, stride=stride)
        assert np.allclose(r["mean"], pts, rtol=0, atol=1e-14) and np.all(r["se"] < 1e-14)
        assert np.all(r["plain_se"] > 1e-3)
        d = W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_SIN)
        r = oracle_mod.fk_solve_cv(W.CONST, d, pts, 0.05, 2e-3, 400, seed=1, uhat=oracle_mod.UHAT_SIN,
                                   stride=stride)
        exact = math.exp(-2 * math.pi ** 2 * 0.05) * np.sin(math.pi * pts[:, 0]) * np.sin(math.pi * pts[:, 1])
        assert np.allclose(r["mean"][:, 0], exact, rtol=0, atol=1e-13) and np.all(r["se"] < 1e-13)


def test_linear_uhat_is_unbiased_with_drift(oracle_mod):
    pts = np.array([[0.35, 0.55], [0.25, 0.62], [0.5, 0.5]])
    r = oracle_mod.fk_solve_cv(W.static_bump(), W.Data(), pts, 0.03, 1e-4, 20000, seed=4,
                               uhat=oracle_mod.UHAT_LINEAR)
    d = np.abs(r["mean"] - r["plain_mean"])
    assert np.all(d <= 3 * np.sqrt(r["se"] ** 2 + r["plain_se"] ** 2))
    # near the bump the CV removes the Brownian part: much lower variance
    assert np.all(r["se"][:2] < 0.5 * r["plain_se"][:2])


def test_network_uhat_agrees_with_plain(oracle_mod):
    flat = M.bf16_round(W.mlp_init(0))
    pts = np.array([[0.5, 0.3], [0.45, 0.6]])
    r = oracle_mod.fk_solve_cv(W.moving_bump(), W.Data(), pts, 0.01, 1e-4, 400, seed=2,
                               uhat=oracle_mod.UHAT_MLP, flat=flat, t_scale=W.CV_T_SCALE, stride=2)
    d = np.abs(r["mean"] - r["plain_mean"])
    assert np.all(d <= 3 * np.sqrt(r["se"] ** 2 + r["plain_se"] ** 2) + 1e-3)
