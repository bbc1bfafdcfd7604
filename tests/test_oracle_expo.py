"""Pins of exponential time-stepping (score mode EXPONENTIAL: step lengths
exponentially distributed with mean dt, the last one cut at the horizon;
Euler-Maruyama given the length; the Brownian-bridge exit test given it).

For w = 1 every step is exact in law given its length, and the bridge test
is exact given it, so the closed forms of the bridge pins hold for random
step lengths too -- at mean steps as coarse as the horizon:

* survival near one side: erf(d / (2 sqrt(t)));
* the decaying sine mode with zero boundary data;
* identity data: E[xi] = x, E[eta] = y (near one side).

The law of the step lengths: a path that does not exit takes 1 + Poisson(t
/ dt) steps (mean and variance pinned far from the boundary).  And with a
moving density the scheme converges to the same values as the fixed-step
bridge scheme (the density's time along a path follows the elapsed random
time).
"""
import math
import os

import numpy as np
import pytest

import workloads as W

THREADS = min(8, os.cpu_count() or 1)
ONES = np.ones((2, 2))


@pytest.mark.parametrize("mean_steps", [1, 4])
def test_survival_near_one_side(oracle_mod, mean_steps):
    t = 1e-3
    d = np.array([0.01, 0.03, 0.05, 0.08])
    pts = np.stack([d, np.full_like(d, 0.5)], 1)
    exact = np.array([math.erf(v / (2 * math.sqrt(t))) for v in d])
    data = W.Data(init_kind=W.DATA_GRID, bdry_kind=W.DATA_ZERO, score_mode=W.SCORE_EXPONENTIAL, grid_xi=ONES,
                  grid_eta=ONES)
    o = oracle_mod.fk_solve(W.CONST, data, pts, t, t / mean_steps, 40000, seed=5 + mean_steps, threads=THREADS)
    z = (o["mean"][:, 0] - exact) / o["se"][:, 0]
    assert np.all(np.abs(z) < 4.5), z
    # without the bridge test the same random steps miss most crossings
    proj = oracle_mod.fk_solve(W.CONST, W.Data(init_kind=W.DATA_GRID, bdry_kind=W.DATA_ZERO,
                                               score_mode=W.SCORE_PROJECT, grid_xi=ONES, grid_eta=ONES),
                               pts, t, t / mean_steps, 40000, seed=5 + mean_steps, threads=THREADS)
    assert ((proj["mean"][:, 0] - exact) / proj["se"][:, 0]).max() > 20


@pytest.mark.parametrize("mean_steps", [1, 5])
def test_sine_mode_exact_at_coarse_steps(oracle_mod, mean_steps):
    t = 0.01
    pts = np.array([[0.05, 0.5], [0.5, 0.93], [0.1, 0.12], [0.3, 0.7], [0.97, 0.4]])
    exact = math.exp(-2 * math.pi ** 2 * t) * np.sin(math.pi * pts[:, 0]) * np.sin(math.pi * pts[:, 1])
    data = W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_ZERO, score_mode=W.SCORE_EXPONENTIAL)
    o = oracle_mod.fk_solve(W.CONST, data, pts, t, t / mean_steps, 40000, seed=17 + mean_steps, threads=THREADS)
    z = (o["mean"][:, 0] - exact) / o["se"][:, 0]
    assert np.all(np.abs(z) < 4.5), z


def test_identity_data_is_unbiased(oracle_mod):
    """Near one side at a time (near a corner the four sides' crossings are
    not independent, for this scheme as for the fixed-step bridge test)."""
    t = 4e-3
    pts = np.array([[0.03, 0.5], [0.5, 0.04], [0.96, 0.45], [0.55, 0.97], [0.08, 0.3]])
    data = W.Data(score_mode=W.SCORE_EXPONENTIAL)
    o = oracle_mod.fk_solve(W.CONST, data, pts, t, t / 2, 40000, seed=23, want_exit=True, threads=THREADS)
    z = (o["mean"] - pts) / o["se"]
    assert np.all(np.abs(z) < 4.5), z
    assert np.mean(o["exit_step"] >= 1) > 0.05          # the boundary is really reached


def test_step_count_law(oracle_mod):
    """Far from the boundary (no exits): steps = 1 + Poisson(t / dt)."""
    t, dt, n_nodes = 2e-3, 1e-4, 4000
    lam = t / dt
    pts = np.full((n_nodes, 2), 0.5)
    data = W.Data(score_mode=W.SCORE_EXPONENTIAL)
    o = oracle_mod.fk_solve(W.CONST, data, pts, t, dt, 2, seed=3, want_exit=True, threads=THREADS)
    assert np.all(o["exit_step"] == -1)
    per_node = o["steps"].astype(np.float64)          # two paths per node
    mean, var = per_node.mean(), per_node.var(ddof=1)
    assert abs(mean - 2 * (1 + lam)) < 4 * math.sqrt(2 * lam / n_nodes)
    # the variance of a sum of two Poisson(lam): 2 lam (a sample variance's
    # standard error is about var sqrt(2 / n))
    assert abs(var - 2 * lam) < 4 * 2 * lam * math.sqrt(2 / n_nodes)
    # the fixed-step scheme takes exactly t / dt steps per path
    f = oracle_mod.fk_solve(W.CONST, W.Data(score_mode=W.SCORE_BRIDGE), pts[:10], t, dt, 2, seed=3, threads=THREADS)
    assert np.all(f["steps"] == 2 * round(lam))


def test_agrees_with_the_fixed_step_bridge_scheme_for_a_moving_density(oracle_mod):
    """Both schemes converge to the same values (weak error O(dt) each);
    a density evaluated at the wrong time along the path would separate
    them by far more than this bound."""
    dens = W.moving_bump()
    pts = np.array([[0.3, 0.4], [0.6, 0.55], [0.45, 0.25]])
    t, dt = 0.05, 5e-5
    e = oracle_mod.fk_solve(dens, W.Data(score_mode=W.SCORE_EXPONENTIAL), pts, t, dt, 20000, seed=31,
                            threads=THREADS)
    f = oracle_mod.fk_solve(dens, W.Data(score_mode=W.SCORE_BRIDGE), pts, t, dt, 20000, seed=32, threads=THREADS)
    se = np.hypot(e["se"], f["se"])
    assert np.all(np.abs(e["mean"] - f["mean"]) < 4 * se + 2e-4), (e["mean"] - f["mean"]) / se
    # the same density over another time window (t_init shifted by -2t) is
    # a different field: the estimates separate, so the agreement above
    # does not hold for just any time argument
    wrong = oracle_mod.fk_solve(W.moving_bump(W.TIME_BACKWARD), W.Data(score_mode=W.SCORE_EXPONENTIAL,
                                                                      t_init=-2 * t), pts, t, dt, 20000, seed=31,
                                threads=THREADS)
    assert np.any(np.abs(wrong["mean"] - f["mean"]) > 8 * se)
