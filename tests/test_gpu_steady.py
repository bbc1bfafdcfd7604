"""The elliptic (steady) variant on the GPU (eq. (2)) against the oracle:
steady sub-domain solves (FP64 round-off) and the one-shot steady mesh --
the elliptic interface solve on the same counters (the Monte-Carlo
contract), then the steady sub-domain solves from the GPU's interface
values, and the mesh's quality against the global steady solve."""
import os

import numpy as np
import pytest

import oracle.mesh_step as MS
import oracle.subdomain as S
import workloads as W
from parity import assert_parity

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)


def cuda(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("px,m,dens,bdry", [
    (4, 8, W.static_bump(), "identity"),
    (2, 20, W.paper_ring(W.TIME_FROZEN, 0.0), "equidistributed"),
    (8, 96, W.two_bumps(W.TIME_FROZEN, 0.05), "identity"),
    (3, 10, W.ridge(), "equidistributed"),
])
def test_steady_subdomain_against_oracle(fk, px, m, dens, bdry):
    import torch
    N = px * m
    x = np.arange(N + 1) / N
    X, Y = np.meshgrid(x, x)
    ij = S.interface_index(px, m)
    rng = np.random.default_rng(N)
    ix = X[ij[:, 1], ij[:, 0]] + 1e-3 * rng.standard_normal(len(ij))
    iy = Y[ij[:, 1], ij[:, 0]] + 1e-3 * rng.standard_normal(len(ij))
    print(f"[gpu] steady subdomain px={px} m={m} kind={dens.kind} bdry={bdry}", flush=True)
    gx, gy = fk.subdomain_solve(dens, 0.0, float("inf"), px, m, None, None, cuda(ix), cuda(iy),
                                bdry_kind=0 if bdry == "identity" else 4)
    torch.cuda.synchronize()
    ox, oy = S.subdomain_be_step(dens, 0.0, np.inf, px, m, None, None, ix, iy, bdry=bdry)
    err = max(np.abs(gx.cpu().numpy() - ox).max(), np.abs(gy.cpu().numpy() - oy).max())
    print(f"max |gpu - oracle| = {err:.3e}", flush=True)
    assert err < 1e-11


def test_steady_mesh_against_oracle(fk, oracle_mod):
    """The static bump (A = 10, s2 = 0.01 at (0.3, 0.6)) on 2 x 2
    sub-domains of a 32-cell grid: every path leaves the square well before
    the horizon."""
    import torch
    from paper_1402_0266_amd.mesh_run import interface_nodes, steady_mesh
    px, m, n_paths, dt, horizon = 2, 16, 2048, 1e-4, 3.0
    dens = W.static_bump()
    print(f"[gpu] steady mesh px={px} m={m} N={n_paths}", flush=True)
    g = steady_mesh(dens, px, m, n_paths, dt, horizon)
    torch.cuda.synchronize()
    assert int(g["survivors"]) == 0
    sx, sy = MS.steady_start(px, m, "identity", dens)
    assert np.abs(g["start"][0].cpu().numpy() - sx).max() < 1e-15
    data = W.Data(init_kind=W.DATA_GRID, bdry_kind=W.DATA_GRID, score_mode=W.SCORE_BRIDGE, grid_xi=sx, grid_eta=sy)
    pts = interface_nodes(px, m)
    o = oracle_mod.fk_solve(dens, data, pts, horizon, dt, n_paths, want_exit=True, want_scores=True,
                            threads=THREADS)
    gg = fk.fk_interface_solve(dens, data, pts, horizon, dt, n_paths, exit_step=True, scores=True,
                               grids=(cuda(sx).view(-1), cuda(sy).view(-1)))
    torch.cuda.synchronize()
    gg = {k: v.cpu().numpy() for k, v in gg.items() if not k.startswith("_")}
    assert np.array_equal(gg["xi"], g["iface_xi"].cpu().numpy())       # the driver's solve is this one
    assert_parity(gg, o, pts, shifted=False, label="steady interface:")
    ix, iy = g["iface_xi"].cpu().numpy(), g["iface_eta"].cpu().numpy()
    ox, oy = S.subdomain_be_step(dens, 0.0, np.inf, px, m, None, None, ix, iy)
    gx, gy = g["xi"].cpu().numpy(), g["eta"].cpu().numpy()
    assert max(np.abs(gx - ox).max(), np.abs(gy - oy).max()) < 1e-11
    # the decomposed steady mesh against the global steady solve, with enough
    # paths that the interface noise (2 SE / h on a cell's Jacobian) stays
    # near 5%
    print("[gpu] steady mesh at 2^17 paths", flush=True)
    g2 = steady_mesh(dens, px, m, 1 << 17, dt, horizon, seed=1)
    torch.cuda.synchronize()
    N = px * m
    fx, fy = S.global_be_step(dens, 0.0, np.inf, N, None, None)
    jd, sd = S.mesh_quality(g2["xi"].cpu().numpy(), g2["eta"].cpu().numpy())
    jg, sg = S.mesh_quality(fx, fy)
    print(f"steady mesh: min J {jd:.4f} (global {jg:.4f}), max skew {sd:.4f} (global {sg:.4f}), "
          f"max se {float(g2['se_xi'].max()):.2e}", flush=True)
    assert int(g2["survivors"]) == 0
    assert jd > 0 and abs(jd - jg) <= 0.1 * jg and abs(sd - sg) <= 0.05
