"""The Brownian-bridge exit test on the GPU (score mode BRIDGE) against the
oracle on the same counters (exit steps, means within 3 SE and 1e-5, SE
within 1%), the closed form it makes exact at a single step, and the test
inside the martingale control-variate kernels (network and mesh gradient)."""
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


def test_martingale_network_form_with_bridge_against_oracle(fk, oracle_mod):
    """The bridge test inside the martingale control-variate kernel: the
    plain part is the plain bridge scheme (same exits), the CV scores are the
    oracle's on the same BF16 weights (BF16 activations: ~1e-2 of the
    martingale sum), the means within 3 SE and 1e-5."""
    import torch
    cv = fk.FkCv(W.mlp_init(7), W.CV_T_SCALE)
    _, bf = cv.params()
    dens = W.moving_bump()
    pts = W.interface_nodes(4, 4, 16)[::3]
    data = W.Data(score_mode=W.SCORE_BRIDGE)
    t, dt, N = 0.01, 2e-4, 1024
    print(f"[gpu] bridge in the martingale form nodes={len(pts)} N={N}", flush=True)
    g = fk.fk_interface_solve_cv(dens, data, pts, t, dt, N, cv, stride=10, seed=3, form=fk.FK_CV_MARTINGALE,
                                 exit_step=True, cv_scores=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}
    o = oracle_mod.fk_solve_cv(dens, data, pts, t, dt, N, seed=3, uhat=oracle_mod.UHAT_MLP, flat=bf,
                               t_scale=W.CV_T_SCALE, stride=10, form=oracle_mod.CV_MARTINGALE, want_scores=True,
                               want_exit=True, threads=THREADS)
    plain = {"xi": g["plain_xi"], "eta": g["plain_eta"], "se_xi": g["plain_se_xi"], "se_eta": g["plain_se_eta"],
             "exit_step": g["exit_step"]}
    assert_parity(plain, {"mean": o["plain_mean"], "se": o["plain_se"], "exit_step": o["exit_step"]}, pts,
                  shifted=False, label="plain part:")
    assert np.mean(g["exit_step"] >= 1) > 0.05
    same = g["exit_step"] == o["exit_step"]
    po = oracle_mod.fk_solve(dens, data, pts, t, dt, N, seed=3, want_scores=True, threads=THREADS)["scores"]
    msum = np.abs(po - o["cv_scores"])[same]
    ds = np.abs(g["cv_scores"].astype(np.float64) - o["cv_scores"])[same]
    rel = ds.max(axis=-1) / np.maximum(msum.max(axis=-1), 1e-3)
    d = np.abs(np.stack([g["xi"], g["eta"]], 1) - o["mean"])
    print(f"bridge, martingale: max rel {rel.max():.2e}, max |mean diff| {d.max():.2e}", flush=True)
    assert rel.max() < 0.05
    assert np.all(d <= 3 * o["se"]) and np.all(d <= 1e-5)
    cv.close()


def test_grid_control_with_bridge_against_oracle(fk, oracle_mod):
    """The mesh-gradient control with the bridge test, grid boundary data at
    the projected exit point: a deformed mesh under two frozen bumps."""
    import torch
    n = 48
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x)
    gx = X + 0.02 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    gy = Y + 0.015 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    dens = W.two_bumps(W.TIME_FROZEN, 0.0375)
    data = W.Data(init_kind=W.DATA_GRID, bdry_kind=W.DATA_GRID, score_mode=W.SCORE_BRIDGE, t_init=0.0375,
                  grid_xi=gx.ravel(), grid_eta=gy.ravel())
    nodes = W.interface_nodes(4, 4, 48)
    pts = np.concatenate([nodes[::7], nodes[np.minimum(nodes, 1 - nodes).min(1) < 0.05][::3]])
    t, dt, N = 5e-4, 2.5e-5, 2048
    print(f"[gpu] bridge with the grid control nodes={len(pts)} N={N}", flush=True)
    g = fk.fk_interface_solve_cv(dens, data, pts, t, dt, N, None, stride=2, seed=5, level_id=2,
                                 form=fk.FK_CV_MARTINGALE_GRID, exit_step=True, cv_scores=True,
                                 grids=(cuda(gx).view(-1), cuda(gy).view(-1)))
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}
    o = oracle_mod.fk_solve_cv(dens, data, pts, t, dt, N, seed=5, level_id=2, uhat=oracle_mod.UHAT_GRID, stride=2,
                               form=oracle_mod.CV_MARTINGALE, want_scores=True, want_exit=True, threads=THREADS)
    plain = {"xi": g["plain_xi"], "eta": g["plain_eta"], "se_xi": g["plain_se_xi"], "se_eta": g["plain_se_eta"],
             "exit_step": g["exit_step"]}
    assert_parity(plain, {"mean": o["plain_mean"], "se": o["plain_se"], "exit_step": o["exit_step"]}, pts,
                  shifted=False, label="plain part:")
    same = g["exit_step"] == o["exit_step"]
    ds = np.abs(g["cv_scores"].astype(np.float64) - o["cv_scores"])[same]
    d = np.abs(np.stack([g["xi"], g["eta"]], 1) - o["mean"])
    print(f"bridge, grid control: max |score diff| {ds.max():.2e}, max |mean diff| {d.max():.2e}", flush=True)
    assert np.mean(ds.max(axis=-1) < 1e-6) >= 0.999 and ds.max() < 1e-3
    assert np.all(d <= 3 * o["se"]) and np.all(d <= 1e-5)


def test_bridge_is_rejected_by_the_dynkin_form(fk):
    cv = fk.FkCv(W.mlp_init(7), W.CV_T_SCALE)
    with pytest.raises(fk.FkError) as e:
        fk.fk_interface_solve_cv(W.CONST, W.Data(score_mode=W.SCORE_BRIDGE), np.array([[0.5, 0.5]]), 0.01, 1e-3,
                                 64, cv, form=fk.FK_CV_DYNKIN)
    assert e.value.code == -5
    cv.close()


def test_short_horizon_bridge_without_a_step_count(fk):
    """Regression: a short horizon (K <= 64) with the bridge test and no
    step-count output (the plain pass of a control-variate solve, or a C
    caller passing NULL) -- the bridge kernel skips the null count, and the
    estimates equal those of the same solve with the count."""
    import ctypes

    import torch
    pts = torch.tensor(W.STATIC_BUMP_31.nodes(), device="cuda")
    n = pts.shape[0]
    data = W.Data(score_mode=W.SCORE_BRIDGE)
    ref = fk.fk_interface_solve(W.static_bump(), data, pts, 2e-3, 1e-4, 2048, 5)
    out = {k: torch.empty(n, dtype=torch.float64, device="cuda") for k in ("xi", "eta", "se_xi", "se_eta")}
    ws = torch.empty(fk.fk_interface_workspace_bytes(n, 2048), dtype=torch.uint8, device="cuda")
    print("[gpu] bridge, K = 20, no step count", flush=True)
    rc = fk.library().fk_interface_solve(
        ctypes.byref(fk._density(W.static_bump())), ctypes.byref(fk._data(data)), pts.data_ptr(), None, n, 2e-3,
        1e-4, 2048, 5, 0, out["xi"].data_ptr(), out["eta"].data_ptr(), out["se_xi"].data_ptr(),
        out["se_eta"].data_ptr(), None, None, None, None, None, ws.data_ptr(), ws.numel(),
        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, fk.fk_last_error()
    torch.cuda.synchronize()
    for k in ("xi", "eta", "se_xi", "se_eta"):
        assert torch.equal(out[k], ref[k]), k
