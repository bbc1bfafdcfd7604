"""The Brownian-bridge exit test on the GPU (score mode BRIDGE) against the
oracle on the same counters (exit steps, means within 3 SE and 1e-5, SE
within 1%), and the closed form it makes exact at a single step."""
import math
import os

import numpy as np
import pytest

import workloads as W
from parity import assert_parity

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)
ONES = np.ones((2, 2))


def cuda(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def run_pair(fk, oracle_mod, dens, data, pts, t, dt, n, seed=0, grids=None, dens_o=None):
    import torch
    print(f"[gpu] bridge kind={dens.kind} nodes={len(pts)} N={n} t={t} dt={dt}", flush=True)
    g = fk.fk_interface_solve(dens, data, pts, t, dt, n, seed, 0, exit_step=True, scores=True, steps=True,
                              grids=None if grids is None else tuple(cuda(x).view(-1) for x in grids))
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}
    o = oracle_mod.fk_solve(dens_o or dens, data, pts, t, dt, n, seed, 0, want_exit=True, want_scores=True,
                            threads=THREADS)
    return g, o


def test_survival_closed_form_one_step(fk, oracle_mod):
    t = 1e-3
    d = np.array([0.01, 0.03, 0.05, 0.08])
    pts = np.stack([d, np.full_like(d, 0.5)], 1)
    data = W.Data(init_kind=W.DATA_GRID, bdry_kind=W.DATA_ZERO, score_mode=W.SCORE_BRIDGE, grid_xi=ONES,
                  grid_eta=ONES)
    g, o = run_pair(fk, oracle_mod, W.CONST, data, pts, t, t, 40000, grids=(ONES, ONES))
    assert_parity(g, o, pts, shifted=False, label="survival:")
    exact = np.array([math.erf(v / (2 * math.sqrt(t))) for v in d])
    z = (g["xi"] - exact) / g["se_xi"]
    assert np.all(np.abs(z) < 4.5), z


@pytest.mark.parametrize("t,dt", [(0.01, 1e-3), (0.0105, 1e-3)])      # the second with a short last step
def test_sine_mode_parity(fk, oracle_mod, t, dt):
    pts = W.uniform_points(24, seed=5, lo=0.0, hi=1.0)
    data = W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_ZERO, score_mode=W.SCORE_BRIDGE)
    g, o = run_pair(fk, oracle_mod, W.CONST, data, pts, t, dt, 8192, seed=2)
    assert_parity(g, o, pts, shifted=False, label="sine mode:")


def test_static_bump_parity(fk, oracle_mod):
    wl = W.STATIC_BUMP_31
    pts = wl.nodes()
    data = W.Data(score_mode=W.SCORE_BRIDGE)
    g, o = run_pair(fk, oracle_mod, wl.density, data, pts, wl.t, wl.dt, 4096)
    assert_parity(g, o, pts, shifted=False, label="static bump:")
    assert np.mean(g["exit_step"] >= 0) > 0.2


def test_moving_bump_subset_parity(fk, oracle_mod):
    wl = W.MOVING_BUMP_1521
    pts = wl.nodes()[::48]
    data = W.Data(score_mode=W.SCORE_BRIDGE)
    g, o = run_pair(fk, oracle_mod, wl.density, data, pts, wl.t, wl.dt, 256)
    assert_parity(g, o, pts, shifted=False, label="moving bump:")


def test_ring_grid_boundary_parity(fk, oracle_mod):
    """The paper's ring sampled on its 41 x 41 grid, a perturbed mesh as
    grid initial data whose edge nodes are the boundary data (FK_DATA_GRID
    boundary data at the projected exit point)."""
    n = 40
    w = oracle_mod.sample_density(W.paper_ring(W.TIME_FROZEN, 0.1), 0.1, n)
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x)
    xi0 = X + 0.01 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    eta0 = Y + 0.01 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    data = W.Data(init_kind=W.DATA_GRID, bdry_kind=W.DATA_GRID, score_mode=W.SCORE_BRIDGE, t_init=0.1,
                  grid_xi=xi0, grid_eta=eta0)
    pts = W.interface_nodes(2, 2, n)
    g, o = run_pair(fk, oracle_mod, fk.GridDensity(cuda(w)), data, pts, 1e-3, 5e-5, 8192, seed=9,
                    grids=(xi0, eta0), dens_o=W.Density(W.KIND_GRID, w_grid=w))
    assert_parity(g, o, pts, shifted=False, label="ring, grid boundary data:")


def test_bridge_is_rejected_by_the_cv_solve(fk):
    with pytest.raises(fk.FkError) as e:
        fk.fk_interface_solve_cv(W.CONST, W.Data(score_mode=W.SCORE_BRIDGE), np.array([[0.5, 0.5]]), 0.01, 1e-3,
                                 64, None, form=fk.FK_CV_MARTINGALE_GRID)
    assert e.value.code in (-1, -5)
