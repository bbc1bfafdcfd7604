"""Pins of the Brownian-bridge exit test (score mode BRIDGE).

For w = 1 the Euler-Maruyama chain is exact in law at the step times, and
the bridge crossing probability exp(-d0 d1 / D) of a straight side is exact
for the pinned diffusion sqrt(2) W; the x and y motions are independent.  So
with the bridge test the killed chain has the law of the killed diffusion
for any step size (up to the product of the two barriers of one coordinate,
~exp(-1/D)), which fixes closed forms at coarse steps:

* survival probability near one side: erf(d / (2 sqrt(t))) (grid initial
  data 1, boundary data 0), at one step and at four and sixteen steps --
  where the discrete test alone (PROJECT) overestimates it by many standard
  errors;
* the decaying sine mode with zero boundary data: exp(-2 pi^2 t) phi(P) at
  one and four steps;
* identity data: E[xi] = x and E[eta] = y (an exit is scored at the exact
  normal coordinate of the crossing; the tangential end point has the right
  mean because the two motions are independent).
"""
import math
import os

import numpy as np
import pytest

import workloads as W

THREADS = min(8, os.cpu_count() or 1)
ONES = np.ones((2, 2))


@pytest.mark.parametrize("steps", [1, 4, 16])
def test_survival_near_one_side(oracle_mod, steps):
    t = 1e-3
    d = np.array([0.01, 0.03, 0.05, 0.08])
    pts = np.stack([d, np.full_like(d, 0.5)], 1)
    exact = np.array([math.erf(v / (2 * math.sqrt(t))) for v in d])
    data = W.Data(init_kind=W.DATA_GRID, bdry_kind=W.DATA_ZERO, score_mode=W.SCORE_BRIDGE, grid_xi=ONES,
                  grid_eta=ONES)
    o = oracle_mod.fk_solve(W.CONST, data, pts, t, t / steps, 40000, seed=steps, threads=THREADS)
    z = (o["mean"][:, 0] - exact) / o["se"][:, 0]
    assert np.all(np.abs(z) < 4.5), z
    if steps == 1:
        proj = oracle_mod.fk_solve(W.CONST, W.Data(init_kind=W.DATA_GRID, bdry_kind=W.DATA_ZERO,
                                                   score_mode=W.SCORE_PROJECT, grid_xi=ONES, grid_eta=ONES),
                                   pts, t, t, 40000, seed=steps, threads=THREADS)
        zp = (proj["mean"][:, 0] - exact) / proj["se"][:, 0]
        assert zp.max() > 20, zp


@pytest.mark.parametrize("steps", [1, 4])
def test_sine_mode_exact_at_coarse_steps(oracle_mod, steps):
    t = 0.01
    pts = np.array([[0.05, 0.5], [0.5, 0.93], [0.1, 0.12], [0.3, 0.7], [0.97, 0.4]])
    exact = math.exp(-2 * math.pi ** 2 * t) * np.sin(math.pi * pts[:, 0]) * np.sin(math.pi * pts[:, 1])
    data = W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_ZERO, score_mode=W.SCORE_BRIDGE)
    o = oracle_mod.fk_solve(W.CONST, data, pts, t, t / steps, 40000, seed=11 + steps, threads=THREADS)
    z = (o["mean"][:, 0] - exact) / o["se"][:, 0]
    assert np.all(np.abs(z) < 4.5), z
    if steps == 1:
        proj = oracle_mod.fk_solve(W.CONST, W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_ZERO,
                                                   score_mode=W.SCORE_PROJECT),
                                   pts, t, t, 40000, seed=11 + steps, threads=THREADS)
        zp = (proj["mean"][:, 0] - exact) / proj["se"][:, 0]
        assert zp.max() > 8, zp


def test_identity_data_is_unbiased(oracle_mod):
    t = 4e-3
    pts = np.array([[0.03, 0.5], [0.5, 0.04], [0.96, 0.45], [0.55, 0.97], [0.08, 0.3]])
    data = W.Data(score_mode=W.SCORE_BRIDGE)
    o = oracle_mod.fk_solve(W.CONST, data, pts, t, t / 2, 40000, seed=3, want_exit=True, threads=THREADS)
    z = (o["mean"] - pts) / o["se"]
    assert np.all(np.abs(z) < 4.5), z
    assert np.mean(o["exit_step"] >= 1) > 0.05          # the boundary is really reached
