"""Exponential time-stepping on the GPU (score mode EXPONENTIAL) against the
oracle on the same counters: exit steps, means within 3 SE and 1e-5, SE
within 1%, the steps taken per node; the w = 1 closed form at a mean step
as coarse as the horizon; a zero horizon; schedule invariance."""
import math
import os

import numpy as np
import pytest

import workloads as W
from parity import assert_parity

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)


def cuda(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def run_pair(fk, oracle_mod, dens, data, pts, t, dt, n, seed=0, grids=None, dens_o=None, level_id=0):
    import torch
    print(f"[gpu] exponential steps kind={dens.kind} nodes={len(pts)} N={n} t={t} dt={dt}", flush=True)
    g = fk.fk_interface_solve(dens, data, pts, t, dt, n, seed, level_id, exit_step=True, scores=True, steps=True,
                              grids=None if grids is None else tuple(cuda(x).view(-1) for x in grids))
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}
    o = oracle_mod.fk_solve(dens_o or dens, data, pts, t, dt, n, seed, level_id, want_exit=True, want_scores=True,
                            threads=THREADS)
    # the steps each node's paths took: random, identical but for rare FP32 /
    # FP64 ties where a step ends at the horizon (checked here instead of
    # exactly in assert_parity)
    assert np.all(np.abs(g["steps"] - o["steps"]) <= 1e-4 * o["steps"] + 2)
    assert int(g["total_steps"][0]) == int(g["steps"].sum())
    return g, o


@pytest.mark.parametrize("mean_steps", [1, 8])
def test_sine_mode_closed_form_and_parity(fk, oracle_mod, mean_steps):
    t = 0.01
    pts = np.array([[0.05, 0.5], [0.5, 0.93], [0.1, 0.12], [0.3, 0.7], [0.97, 0.4]])
    data = W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_ZERO, score_mode=W.SCORE_EXPONENTIAL)
    g, o = run_pair(fk, oracle_mod, W.CONST, data, pts, t, t / mean_steps, 20000, seed=mean_steps)
    assert_parity(g, o, pts, shifted=False, label=f"sine mode, mean {mean_steps} steps:", exact_steps=False)
    exact = math.exp(-2 * math.pi ** 2 * t) * np.sin(math.pi * pts[:, 0]) * np.sin(math.pi * pts[:, 1])
    assert np.all(np.abs(g["xi"] - exact) < 4.5 * g["se_xi"])


def test_static_bump_parity(fk, oracle_mod):
    wl = W.STATIC_BUMP_31
    pts = wl.nodes()
    g, o = run_pair(fk, oracle_mod, wl.density, W.Data(score_mode=W.SCORE_EXPONENTIAL), pts, wl.t, wl.dt, 4096)
    assert_parity(g, o, pts, shifted=False, label="static bump:", exact_steps=False)
    assert np.mean(g["exit_step"] >= 0) > 0.2


def test_moving_bump_subset_parity(fk, oracle_mod):
    """A density moving on its orbit: its time follows each path's own
    random elapsed time."""
    wl = W.MOVING_BUMP_1521
    pts = wl.nodes()[::48]
    g, o = run_pair(fk, oracle_mod, wl.density, W.Data(score_mode=W.SCORE_EXPONENTIAL), pts, 0.02, 1e-4, 512,
                    seed=4, level_id=3)
    assert_parity(g, o, pts, shifted=False, label="moving bump:", exact_steps=False)


def test_ring_grid_boundary_parity(fk, oracle_mod):
    n = 40
    w = oracle_mod.sample_density(W.paper_ring(W.TIME_FROZEN, 0.1), 0.1, n)
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x)
    xi0 = X + 0.01 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    eta0 = Y + 0.01 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    data = W.Data(init_kind=W.DATA_GRID, bdry_kind=W.DATA_GRID, score_mode=W.SCORE_EXPONENTIAL, t_init=0.1,
                  grid_xi=xi0, grid_eta=eta0)
    pts = W.interface_nodes(2, 2, n)
    g, o = run_pair(fk, oracle_mod, fk.GridDensity(cuda(w)), data, pts, 1e-3, 5e-5, 8192, seed=9,
                    grids=(xi0, eta0), dens_o=W.Density(W.KIND_GRID, w_grid=w))
    assert_parity(g, o, pts, shifted=False, label="ring, grid boundary data:", exact_steps=False)


def test_zero_horizon_and_schedule_invariance(fk):
    import torch
    pts = np.array([[0.3, 0.4], [0.9, 0.05]])
    data = W.Data(score_mode=W.SCORE_EXPONENTIAL)
    r = fk.fk_interface_solve(W.static_bump(), data, pts, 0.0, 1e-4, 64, steps=True)
    torch.cuda.synchronize()
    assert np.allclose(r["xi"].cpu().numpy(), pts[:, 0], atol=1e-14) and int(r["steps"].sum()) == 0
    a = fk.fk_interface_solve(W.static_bump(), data, pts, 0.01, 1e-4, 3000, 7, scores=True, steps=True)
    b = fk.fk_interface_solve(W.static_bump(), data, pts, 0.01, 1e-4, 3000, 7, scores=True, steps=True,
                              plan={"block": 64, "chunk": 7, "blocks_per_cu": 2})
    torch.cuda.synchronize()
    for k in ("xi", "eta", "se_xi", "se_eta", "scores", "steps"):
        assert np.array_equal(a[k].cpu().numpy(), b[k].cpu().numpy()), k
