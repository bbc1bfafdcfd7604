"""Key points and interface interpolation on the GPU (Sect. 4 speed-up;
Sect. 5) against the oracle:

* the key-point mask, bit for bit, from the same samples of w (both sides
  take every decision in FP64 from sums and differences only);
* the interpolated interface values (FP64 round-off);
* the outer boundary data of a mesh step (identity and equidistributed);
* the paper's run with key points, step by step: mask, key estimates (the
  Monte-Carlo contract on the same counters), interpolated values, mesh.
"""
import math
import os

import numpy as np
import pytest

import oracle.keypoints as K
import oracle.subdomain as S
import workloads as W

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)


def cuda(a, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda")


CASES = [
    (W.paper_ring(W.TIME_FROZEN, 0.0), 0.0, 2, 20, 1e-2, 10),     # the paper's 41 x 41 grid
    (W.paper_ring(W.TIME_FROZEN, 0.0), 0.37, 2, 20, 1e-2, 10),
    (W.two_bumps(W.TIME_FROZEN, 0.0), 0.05, 8, 96, 1e-2, 48),     # the 768-cell run
    (W.moving_bump(), 0.08, 4, 64, 1e-3, 16),
    (W.CONST, 0.0, 3, 10, 1e-2, 3),                              # flat: crossings and gap fill only
]


@pytest.mark.parametrize("dens,tau,px,m,tol,gap", CASES)
def test_key_mask_against_oracle(fk, oracle_mod, dens, tau, px, m, tol, gap):
    import torch
    w = oracle_mod.sample_density(dens, tau, px * m)
    print(f"[gpu] key points kind={dens.kind} tau={tau} px={px} m={m}", flush=True)
    g = fk.fk_key_points(cuda(w), px, m, tol, gap)
    torch.cuda.synchronize()
    o = K.key_mask(w, px, m, tol, gap)
    gm = g.cpu().numpy().astype(bool)
    print(f"keys {int(gm.sum())} of {gm.size}", flush=True)
    assert np.array_equal(gm, o)


@pytest.mark.parametrize("dens,tau,px,m,tol,gap", CASES)
def test_interpolation_against_oracle(fk, oracle_mod, dens, tau, px, m, tol, gap):
    import torch
    N = px * m
    mask = K.key_mask(oracle_mod.sample_density(dens, tau, N), px, m, tol, gap)
    rng = np.random.default_rng(N + m)
    X, Y = np.meshgrid(np.arange(N + 1) / N, np.arange(N + 1) / N)
    ex = X + 0.03 * rng.standard_normal(X.shape)       # arbitrary edge data
    ey = Y + 0.03 * rng.standard_normal(Y.shape)
    pts = S.interface_index(px, m) / N
    keys = pts[mask] + 0.05 * rng.standard_normal((int(mask.sum()), 2))
    slot = np.full(mask.size, -1, dtype=np.int32)
    slot[mask] = np.arange(int(mask.sum()), dtype=np.int32)
    print(f"[gpu] interpolation px={px} m={m} keys={int(mask.sum())}", flush=True)
    gx, gy = fk.fk_interface_interpolate(px, m, cuda(slot, torch.int32), cuda(keys[:, 0]), cuda(keys[:, 1]),
                                         cuda(ex), cuda(ey))
    torch.cuda.synchronize()
    o = K.interpolate_interface(px, m, mask, keys, ex, ey)
    g = np.stack([gx.cpu().numpy(), gy.cpu().numpy()], 1)
    assert np.abs(g - o).max() < 1e-13
    # the in-place form on the mask: key values in their nodes' rows, the
    # rest garbage that must be overwritten; bitwise the slot form's result
    ix = np.full(mask.size, 1e300)
    iy = np.full(mask.size, -1e300)
    ix[mask], iy[mask] = keys[:, 0], keys[:, 1]
    ix, iy = cuda(ix), cuda(iy)
    fk.fk_interface_interpolate_mask(px, m, cuda(mask, torch.uint8), cuda(ex), cuda(ey), ix, iy)
    torch.cuda.synchronize()
    assert np.array_equal(ix.cpu().numpy(), g[:, 0]) and np.array_equal(iy.cpu().numpy(), g[:, 1])


@pytest.mark.parametrize("dens,t_w,n,bdry", [
    (W.paper_ring(W.TIME_FROZEN, 0.2), 0.2, 40, "equidistributed"),
    (W.two_bumps(W.TIME_FROZEN, 0.0), 0.0, 64, "identity"),
    (None, 0.3, 40, "equidistributed"),      # grid density: the sampled ring
])
def test_boundary_data_against_oracle(fk, oracle_mod, dens, t_w, n, bdry):
    import torch
    if dens is None:
        w = oracle_mod.sample_density(W.paper_ring(W.TIME_FROZEN, t_w), t_w, n)
        gdens, odens = fk.GridDensity(cuda(w)), W.Density(W.KIND_GRID, w_grid=w)
    else:
        gdens = odens = dens
    xo = torch.full((n + 1, n + 1), 7.0, dtype=torch.float64, device="cuda")
    yo = torch.full_like(xo, 7.0)
    print(f"[gpu] boundary data n={n} bdry={bdry}", flush=True)
    fk.fk_boundary_data(gdens, t_w, n, 0 if bdry == "identity" else 4, xo, yo)
    torch.cuda.synchronize()
    ox, oy = S.boundary_grid(n, bdry, odens, t_w)
    gx, gy = xo.cpu().numpy(), yo.cpu().numpy()
    edge = np.zeros((n + 1, n + 1), dtype=bool)
    edge[0, :] = edge[-1, :] = edge[:, 0] = edge[:, -1] = True
    assert np.abs(gx[edge] - ox[edge]).max() < 1e-12 and np.abs(gy[edge] - oy[edge]).max() < 1e-12
    assert np.all(gx[~edge] == 7.0) and np.all(gy[~edge] == 7.0)    # the interior is left alone


@pytest.mark.parametrize("density_data", ["analytic", "grid"])
def test_paper_run_with_key_points_against_oracle(fk, oracle_mod, density_data):
    """The paper's run as the paper describes it (Sect. 5): key points on the
    41 x 41 grid, piecewise cubic Hermite interpolation of the other
    interface nodes; three steps against the oracle."""
    import torch
    from paper_1402_0266_amd.mesh_run import PAPER_RING_RUN, MeshRun, MeshRunConfig, paper_ring_density
    cfg = MeshRunConfig(**{**PAPER_RING_RUN, "n_steps": 3, "key_points": True, "density_data": density_data})
    run = MeshRun(cfg, density_fn=paper_ring_density)
    D, N, px, m = cfg.dt_mesh, cfg.px * cfg.m, cfg.px, cfg.m
    for n in range(3):
        xi_n, eta_n = run.mesh()
        tn = n * D
        print(f"[gpu] paper run with key points ({density_data}) step {n}", flush=True)
        run.step()
        torch.cuda.synchronize()
        w = run._wg.cpu().numpy()                          # the driver's samples of w at t^n
        mask = run._mask.cpu().numpy().astype(bool)
        assert np.array_equal(mask, K.key_mask(w, px, m, cfg.key_tol, m // 2))
        assert run.n_keys[n] == int(mask.sum()) < mask.size
        iface, se = run.interface_values()
        ring = W.paper_ring(W.TIME_FROZEN, tn)
        dens = ring if density_data == "analytic" else W.Density(W.KIND_GRID, w_grid=w)
        data = W.Data(init_kind=W.DATA_GRID, score_mode=W.SCORE_EXTEND, t_init=tn, grid_xi=xi_n, grid_eta=eta_n)
        pts = run.pts_host[mask]
        # a masked solve keeps each node's own random stream (its index)
        o = oracle_mod.fk_solve(dens, data, pts, D, D / cfg.substeps, cfg.n_paths, level_id=n,
                                node_ids=np.flatnonzero(mask), threads=THREADS)
        d = np.abs(iface[n][mask] - o["mean"])
        c = (0.5 + 0.25 * math.cos(2 * math.pi * tn), 0.5 + 0.25 * math.sin(2 * math.pi * tn))
        on_ring = np.abs((pts[:, 0] - c[0]) ** 2 + (pts[:, 1] - c[1]) ** 2 - 0.01) < 1e-6
        if density_data == "grid":
            on_ring[:] = False                            # the sampled drift is continuous
        print(f"step {n}: {int(mask.sum())} keys, max |gpu - oracle| {d.max():.2e}, "
              f"max d/se {(d / o['se']).max():.2f}", flush=True)
        assert np.all(d <= 3 * o["se"])
        assert np.all(d[~on_ring] <= 1e-5)
        assert np.all(np.abs(se[n][mask] - o["se"]) <= 0.01 * o["se"])
        gx, gy = run.mesh()
        ib = S.boundary_grid(N, "equidistributed", dens, tn)
        full = K.interpolate_interface(px, m, mask, iface[n][mask], ib[0], ib[1])
        assert np.abs(full - iface[n]).max() < 1e-11     # edge data: quadrature vs Simpson, ~1e-12
        sx, sy = S.subdomain_be_step(dens, tn, D, px, m, xi_n, eta_n, iface[n][:, 0], iface[n][:, 1],
                                     bdry="equidistributed")
        assert np.abs(gx - sx).max() < 1e-11 and np.abs(gy - sy).max() < 1e-11
        q = run.qualities()[n]
        jo, so = S.mesh_quality(gx, gy)
        assert abs(q[0] - jo) < 1e-12 and abs(q[1] - so) < 1e-12 and q[0] > 0
    run.close()
