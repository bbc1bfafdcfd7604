"""The grid data path for w on the GPU (Sect. 4: w known at grid nodes only,
grad w by finite differences, the drift bilinear between the nodes) against
the oracle's independent implementation:

* ``fk_density_sample`` against the oracle's density at the nodes;
* the nodal drift table of ``fk_density_grid_drift`` against the oracle's
  drift at the nodes (FP32 rounding of FP64 values);
* path parity with a grid density (same counters): exit steps, means, SE;
* sub-domain solves with a grid density, equidistributed edges included;
* the paper's run with the grid data path, step by step.
"""
import math
import os

import numpy as np
import pytest

import oracle.subdomain as S
import workloads as W
from parity import assert_parity

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)


def cuda(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def nodal_points(n):
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x)
    return np.stack([X.ravel(), Y.ravel()], 1)


@pytest.mark.parametrize("dens,tau,n", [
    (W.static_bump(), 0.0, 64),
    (W.moving_bump(), 0.13, 40),
    (W.two_bumps(W.TIME_FROZEN, 0.0), 0.07, 96),
    (W.paper_ring(W.TIME_FROZEN, 0.0), 0.3, 40),
    (W.ridge(), 0.0, 17),
    (W.CONST, 0.0, 5),
])
def test_density_sample_against_oracle(fk, oracle_mod, dens, tau, n):
    import torch
    print(f"[gpu] density sample kind={dens.kind} tau={tau} n={n}", flush=True)
    g = fk.fk_density_sample(dens, tau, n)
    torch.cuda.synchronize()
    o = oracle_mod.sample_density(dens, tau, n)
    assert np.abs(g.cpu().numpy() - o).max() <= 1e-14 * np.abs(o).max()


@pytest.mark.parametrize("dens,tau,n", [
    (W.static_bump(), 0.0, 64),
    (W.paper_ring(W.TIME_FROZEN, 0.0), 0.25, 40),
    (W.two_bumps(W.TIME_FROZEN, 0.0), 0.0, 300),
])
def test_drift_table_against_oracle(fk, oracle_mod, dens, tau, n):
    import torch
    w = oracle_mod.sample_density(dens, tau, n)
    print(f"[gpu] drift table kind={dens.kind} n={n}", flush=True)
    b = fk.fk_density_grid_drift(cuda(w))
    torch.cuda.synchronize()
    _, ob = oracle_mod.density(W.Density(W.KIND_GRID, w_grid=w), 0.0, nodal_points(n))
    gb = b.cpu().numpy().reshape(-1, 2).astype(np.float64)
    # FP32 rounding of the FP64 drift (2^-24 relative), and the oracle's
    # bilinear evaluation at the node (~1e-16 relative)
    assert np.all(np.abs(gb - ob) <= 2 ** -24 * np.abs(ob) + 1e-12 * np.abs(ob).max())


def _run_pair(fk, oracle_mod, dens_o, dens_g, data, pts, t, dt, n, seed=0, grids=None):
    import torch
    print(f"[gpu] grid-density solve nodes={len(pts)} N={n} t={t} dt={dt}", flush=True)
    g = fk.fk_interface_solve(dens_g, data, pts, t, dt, n, seed, 0, exit_step=True, scores=True, steps=True,
                              grids=grids)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}
    o = oracle_mod.fk_solve(dens_o, data, pts, t, dt, n, seed, 0, want_exit=True, want_scores=True,
                            threads=THREADS)
    return g, o


def test_sampled_static_bump_paths(fk, oracle_mod):
    """The static-bump workload (31 nodes on x = 1/2, t = 0.05, dt = 1e-4)
    with w sampled on a 256-cell grid."""
    wl = W.STATIC_BUMP_31
    pts = wl.nodes()
    w = oracle_mod.sample_density(wl.density, 0.0, 256)
    g, o = _run_pair(fk, oracle_mod, W.Density(W.KIND_GRID, w_grid=w), fk.GridDensity(cuda(w)), wl.data, pts,
                     wl.t, wl.dt, 4096)
    assert_parity(g, o, pts, label="sampled static bump:")


def test_sampled_ring_paths_with_grid_data(fk, oracle_mod):
    """The paper's ring sampled on its 41 x 41 grid at t = 0.2, the 77
    interface nodes of 2 x 2 sub-domains, a perturbed mesh as grid initial
    data scored past the edge, one mesh step of 1e-3 in 20 sub-steps."""
    n = 40
    w = oracle_mod.sample_density(W.paper_ring(W.TIME_FROZEN, 0.2), 0.2, n)
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x)
    xi0 = X + 0.01 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    eta0 = Y + 0.01 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    data = W.Data(init_kind=W.DATA_GRID, score_mode=W.SCORE_EXTEND, t_init=0.2, grid_xi=xi0, grid_eta=eta0)
    pts = W.interface_nodes(2, 2, n)
    g, o = _run_pair(fk, oracle_mod, W.Density(W.KIND_GRID, w_grid=w), fk.GridDensity(cuda(w)), data, pts,
                     1e-3, 5e-5, 8192, seed=4, grids=(cuda(xi0).view(-1), cuda(eta0).view(-1)))
    assert_parity(g, o, pts, shifted=False, label="sampled ring:")


@pytest.mark.parametrize("px,m,dens,t_w,D,bdry", [
    (2, 20, W.paper_ring(W.TIME_FROZEN, 0.3), 0.3, 1e-3, "equidistributed"),
    (4, 16, W.two_bumps(W.TIME_FROZEN, 0.03), 0.03, 5e-4, "identity"),
    (8, 96, W.two_bumps(W.TIME_FROZEN, 0.05), 0.05, 5e-4, "identity"),
])
def test_subdomain_with_grid_density(fk, oracle_mod, px, m, dens, t_w, D, bdry):
    import torch
    N = px * m
    x = np.arange(N + 1) / N
    X, Y = np.meshgrid(x, x)
    xi0 = X + 0.02 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    eta0 = Y + 0.015 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    ij = S.interface_index(px, m)
    rng = np.random.default_rng(N)
    ix = xi0[ij[:, 1], ij[:, 0]] + 1e-3 * rng.standard_normal(len(ij))
    iy = eta0[ij[:, 1], ij[:, 0]] + 1e-3 * rng.standard_normal(len(ij))
    w = oracle_mod.sample_density(dens, t_w, N)
    kind = 0 if bdry == "identity" else 4
    print(f"[gpu] subdomain with grid density px={px} m={m} bdry={bdry}", flush=True)
    gx, gy = fk.subdomain_solve(fk.GridDensity(cuda(w)), t_w, D, px, m, cuda(xi0), cuda(eta0), cuda(ix), cuda(iy),
                                bdry_kind=kind)
    torch.cuda.synchronize()
    ox, oy = S.subdomain_be_step(W.Density(W.KIND_GRID, w_grid=w), t_w, D, px, m, xi0, eta0, ix, iy, bdry=bdry)
    err = max(np.abs(gx.cpu().numpy() - ox).max(), np.abs(gy.cpu().numpy() - oy).max())
    print(f"max |gpu - oracle| = {err:.3e}", flush=True)
    assert err < 1e-11


def test_paper_run_with_grid_density_against_oracle(fk, oracle_mod):
    """The paper's run with the paper's data path: at each step the ring is
    sampled at t^n on the 41 x 41 mesh grid, and both the interface solve
    and the sub-domain solves take the finite-difference drift.  Three steps
    against the oracle, all 77 interface nodes (the sampled drift is
    continuous, so every node is held to the full contract)."""
    import torch
    from paper_1402_0266_amd import GridDensity, fk_interface_solve
    from paper_1402_0266_amd.mesh_run import PAPER_RING_RUN, GridData, MeshRun, MeshRunConfig, paper_ring_density
    cfg = MeshRunConfig(**{**PAPER_RING_RUN, "n_steps": 3, "density_data": "grid"})
    run = MeshRun(cfg, density_fn=paper_ring_density)
    D, N = cfg.dt_mesh, cfg.px * cfg.m
    for n in range(3):
        xi_n, eta_n = run.mesh()
        tn = n * D
        w = oracle_mod.sample_density(W.paper_ring(W.TIME_FROZEN, tn), tn, N)
        gd = GridDensity(fk.fk_density_sample(paper_ring_density(tn), tn, N))
        g = fk_interface_solve(gd, GridData(t_init=tn, score_mode=cfg.score_mode), run.pts, D, D / cfg.substeps,
                               cfg.n_paths, seed=cfg.seed, level_id=n, exit_step=True, scores=True,
                               grids=(run.xi.view(-1), run.eta.view(-1)))
        print(f"[gpu] paper run (grid density) step {n}", flush=True)
        run.step()
        torch.cuda.synchronize()
        g = {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}
        iface, _ = run.interface_values()
        # the driver's step is the solve above (same samples, same counters)
        assert np.array_equal(iface[n, :, 0], g["xi"]) and np.array_equal(iface[n, :, 1], g["eta"])
        dens = W.Density(W.KIND_GRID, w_grid=w)
        data = W.Data(init_kind=W.DATA_GRID, score_mode=W.SCORE_EXTEND, t_init=tn, grid_xi=xi_n, grid_eta=eta_n)
        o = oracle_mod.fk_solve(dens, data, run.pts_host, D, D / cfg.substeps, cfg.n_paths, level_id=n, want_exit=True,
                                want_scores=True, threads=THREADS)
        assert_parity({k: v for k, v in g.items() if k != "steps"}, o, run.pts_host, shifted=False, label=f"step {n}:")
        sx, sy = S.subdomain_be_step(dens, tn, D, cfg.px, cfg.m, xi_n, eta_n, iface[n, :, 0], iface[n, :, 1],
                                     bdry="equidistributed")
        gx, gy = run.mesh()
        assert np.abs(gx - sx).max() < 1e-11 and np.abs(gy - sy).max() < 1e-11
        q = run.qualities()[n]
        jo, so = S.mesh_quality(gx, gy)
        assert abs(q[0] - jo) < 1e-12 and abs(q[1] - so) < 1e-12 and q[0] > 0
    run.close()
