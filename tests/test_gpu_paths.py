"""GPU parity of the Monte-Carlo interface solve against the FP64 CPU oracle.

Same Philox counters on both sides.  The bar (per node, per component):
  * exit steps identical on >= 99.9% of paths,
  * mean within 3 standard errors AND within 1e-5 absolute of the oracle's
    estimate on the same random stream,
  * standard error within 1% relative.
Plus closed forms that hold for any step size (w = 1 identity data and the
decaying sine mode), invariants, edge cases and schedule invariance.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from parity import assert_parity

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    return torch


def run_gpu(fk, torch, dens, data, pts, t, dt, n, seed=0, level_id=0, plan=None, grids=None):
    print(f"[gpu] kind={dens.kind} mode={dens.time_mode} nodes={len(pts)} N={n} t={t} dt={dt} seed={seed}",
          flush=True)
    g = fk.fk_interface_solve(dens, data, pts, t, dt, n, seed, level_id, exit_step=True, scores=True,
                              steps=True, plan=plan, grids=grids)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}


def run_oracle(oracle_mod, dens, data, pts, t, dt, n, seed=0, level_id=0):
    return oracle_mod.fk_solve(dens, data, pts, t, dt, n, seed, level_id, want_exit=True, want_scores=True,
                               threads=THREADS)


def test_static_bump_31_nodes_full(fk, torch_cuda, oracle_mod):
    """Two sub-domains, 31 interface nodes, t = 0.05, dt = 1e-4, 10^4 paths."""
    wl = W.STATIC_BUMP_31
    pts = wl.nodes()
    g = run_gpu(fk, torch_cuda, wl.density, wl.data, pts, wl.t, wl.dt, wl.n_paths)
    o = run_oracle(oracle_mod, wl.density, wl.data, pts, wl.t, wl.dt, wl.n_paths)
    assert_parity(g, o, pts)
    # invariants: means in [0, 1]; eta non-decreasing along the vertical interface
    m = np.stack([g["xi"], g["eta"]], axis=1)
    s = np.stack([g["se_xi"], g["se_eta"]], axis=1)
    assert np.all(m >= -3 * s) and np.all(m <= 1 + 3 * s)
    de = np.diff(g["eta"])
    assert np.all(de >= -3 * np.sqrt(s[1:, 1] ** 2 + s[:-1, 1] ** 2))


def test_moving_bump_node_subset(fk, torch_cuda, oracle_mod):
    """Moving bump, 4x4 layout, every 32nd canonical node, t = 0.1, dt = 1e-5."""
    wl = W.MOVING_BUMP_1521
    pts = wl.nodes()[::32]
    g = run_gpu(fk, torch_cuda, wl.density, wl.data, pts, wl.t, wl.dt, 512)
    o = run_oracle(oracle_mod, wl.density, wl.data, pts, wl.t, wl.dt, 512)
    assert_parity(g, o, pts)


def test_const_identity_exact(fk, torch_cuda, oracle_mod):
    """w = 1, identity data: the discrete chain is a martingale stopped at the
    exit (unclamped scoring), so E = P exactly for any dt."""
    pts = W.uniform_points(40, seed=1, lo=0.0, hi=1.0)
    g = run_gpu(fk, torch_cuda, W.CONST, W.Data(), pts, 0.08, 2e-3, 4000, seed=3)
    o = run_oracle(oracle_mod, W.CONST, W.Data(), pts, 0.08, 2e-3, 4000, seed=3)
    assert_parity(g, o, pts)
    z = (np.stack([g["xi"], g["eta"]], 1) - pts) / np.stack([g["se_xi"], g["se_eta"]], 1)
    assert np.all(np.abs(z) < 4.5)


def test_const_sin_mode_closed_form(fk, torch_cuda, oracle_mod):
    """w = 1, phi = sin(pi x) sin(pi y), boundary data exp(-2 pi^2 (t-s)) phi:
    E = exp(-2 pi^2 t) phi(P) for any dt."""
    pts = W.uniform_points(24, seed=2)
    data = W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_SIN)
    t, dt = 0.05, 1e-3
    g = run_gpu(fk, torch_cuda, W.CONST, data, pts, t, dt, 8000, seed=5)
    o = run_oracle(oracle_mod, W.CONST, data, pts, t, dt, 8000, seed=5)
    assert_parity(g, o, pts, shifted=False)
    exact = math.exp(-2 * math.pi ** 2 * t) * np.sin(math.pi * pts[:, 0]) * np.sin(math.pi * pts[:, 1])
    assert np.all(np.abs(g["xi"] - exact) <= 4.5 * g["se_xi"] + 1e-12)


def test_ridge_eta_exact(fk, torch_cuda, oracle_mod):
    """w = w(x): the y-drift vanishes, so eta = y exactly for any dt."""
    pts = W.uniform_points(24, seed=4)
    dens = W.ridge()
    g = run_gpu(fk, torch_cuda, dens, W.Data(), pts, 0.05, 1e-4, 4000, seed=7)
    o = run_oracle(oracle_mod, dens, W.Data(), pts, 0.05, 1e-4, 4000, seed=7)
    assert_parity(g, o, pts)
    assert np.all(np.abs(g["eta"] - pts[:, 1]) <= 4.5 * g["se_eta"])


@pytest.mark.parametrize("score_mode", [W.SCORE_PROJECT, W.SCORE_EXTEND])
def test_two_bumps_frozen_grid_data(fk, torch_cuda, oracle_mod, score_mode):
    """Two counter-rotating bumps frozen at t_n, initial data bilinear in a
    nodal grid (one mesh step), exits scored on the projected point or with
    the grid continued past the edge; nodes next to the edges included."""
    import torch
    n = 48
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x)
    gx = X + 0.02 * np.sin(np.pi * X) * np.sin(2 * np.pi * Y)
    gy = Y + 0.02 * np.sin(2 * np.pi * X) * np.sin(np.pi * Y)
    dens = W.two_bumps(W.TIME_FROZEN, t_freeze=0.0375)
    data = W.Data(init_kind=W.DATA_GRID, bdry_kind=W.DATA_IDENTITY, score_mode=score_mode,
                  t_init=0.0375, grid_xi=gx.ravel(), grid_eta=gy.ravel())
    nodes = W.interface_nodes(4, 4, 48)
    near_edge = np.minimum(nodes, 1 - nodes).min(1) < 0.05
    pts = np.concatenate([nodes[::7], nodes[near_edge][::3]])
    grids = (torch.tensor(gx.ravel(), device="cuda"), torch.tensor(gy.ravel(), device="cuda"))
    g = run_gpu(fk, torch_cuda, dens, data, pts, 5e-4, 2.5e-5, 4000, seed=11, grids=grids)
    o = run_oracle(oracle_mod, dens, data, pts, 5e-4, 2.5e-5, 4000, seed=11)
    assert_parity(g, o, pts, shifted=False)


def test_moving_bump_project_and_level_id(fk, torch_cuda, oracle_mod):
    wl = W.MOVING_BUMP_1521
    pts = W.uniform_points(16, seed=6)
    data = W.Data(score_mode=W.SCORE_PROJECT)
    g = run_gpu(fk, torch_cuda, wl.density, data, pts, 0.02, 5e-5, 2000, seed=13, level_id=37)
    o = run_oracle(oracle_mod, wl.density, data, pts, 0.02, 5e-5, 2000, seed=13, level_id=37)
    assert_parity(g, o, pts)


def test_edge_cases(fk, torch_cuda, oracle_mod):
    dens = W.static_bump()
    # no nodes: a valid no-op
    r = fk.fk_interface_solve(dens, W.Data(), np.zeros((0, 2)), 0.05, 1e-4, 16)
    torch_cuda.cuda.synchronize()
    assert r["xi"].numel() == 0
    # t = 0: K = 0, every path scores the initial data at its start point
    pts = np.array([[0.5, 0.25], [0.1, 0.9]])
    g = run_gpu(fk, torch_cuda, dens, W.Data(), pts, 0.0, 1e-4, 64)
    assert np.allclose(g["xi"], pts[:, 0], rtol=0, atol=1e-14)
    assert np.allclose(g["eta"], pts[:, 1], rtol=0, atol=1e-14)
    assert np.all(g["se_xi"] <= 1e-15) and np.all(g["exit_step"] == -1)
    # odd K with a short last step; nodes on the boundary; n_paths = 2
    pts = np.array([[0.0, 0.5], [1.0, 0.3], [0.5, 0.0], [0.37, 1.0], [0.5, 0.5]])
    for n_paths in (2, 333):
        g = run_gpu(fk, torch_cuda, dens, W.Data(), pts, 1.05e-3, 1e-4, n_paths, seed=17)
        o = run_oracle(oracle_mod, dens, W.Data(), pts, 1.05e-3, 1e-4, n_paths, seed=17)
        assert_parity(g, o, pts)


def test_schedule_invariance(fk, torch_cuda):
    """Results depend only on the counters, not on the launch plan: per-path
    records and the fixed-order FP64 reduction are bitwise identical."""
    wl = W.STATIC_BUMP_31
    pts = wl.nodes()
    a = run_gpu(fk, torch_cuda, wl.density, wl.data, pts, wl.t, wl.dt, 3000)
    b = run_gpu(fk, torch_cuda, wl.density, wl.data, pts, wl.t, wl.dt, 3000,
                plan={"block": 64, "chunk": 7, "blocks_per_cu": 3})
    c = run_gpu(fk, torch_cuda, wl.density, wl.data, pts, wl.t, wl.dt, 3000)
    for k in ("xi", "eta", "se_xi", "se_eta", "exit_step", "scores", "steps"):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k
    # a short horizon (20 steps: the default takes 256 paths per grab) and
    # grids cut to the chunk count, down to a single wavefront
    ring = W.paper_ring(W.TIME_FROZEN, 0.3)
    pts = W.interface_nodes(2, 2, 40)
    runs = [run_gpu(fk, torch_cuda, ring, W.Data(), pts, 1e-3, 5e-5, 1000, plan=pl)
            for pl in (None, {"chunk": 128}, {"block": 64, "chunk": 7, "blocks_per_cu": 3}, {"chunk": 1000})]
    one = [run_gpu(fk, torch_cuda, ring, W.Data(), pts[:1], 1e-3, 5e-5, 50, plan=pl)
           for pl in (None, {"chunk": 50})]
    for k in ("xi", "eta", "se_xi", "se_eta", "exit_step", "scores", "steps"):
        for r in runs[1:]:
            assert np.array_equal(runs[0][k], r[k]), k
        assert np.array_equal(one[0][k], one[1][k]), k
    for k in ("exit_step", "scores"):           # the same counters: node 0's first 50 paths
        assert np.array_equal(one[0][k][0], runs[0][k][0][:50]), k
    for r in runs + one:                        # the short form still counts steps when asked
        assert int(r["total_steps"][0]) == int(r["steps"].sum())


def test_in_kernel_estimator_equals_two_pass_fp64(fk, torch_cuda):
    """The estimator is summed inside the path kernel in fixed point; against
    a two-pass FP64 mean and sample variance of the same per-path scores
    (dumped by the kernel) it agrees to 1e-12 relative (means) and 1e-9
    relative (standard errors), and per-node step counts need no per-path
    output."""
    wl = W.MOVING_BUMP_1521
    pts = wl.nodes()[::16]
    for data, t, dt, n in ((wl.data, 0.02, 1e-5, 3000), (W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_SIN),
                                                          0.01, 1e-4, 777)):
        g = run_gpu(fk, torch_cuda, wl.density, data, pts, t, dt, n, seed=5)
        sc = g["scores"].astype(np.float64)
        shift = pts.astype(np.float32).astype(np.float64) if data.init_kind == W.DATA_IDENTITY else 0.0
        mean = sc.mean(axis=1) + shift
        se = sc.std(axis=1, ddof=1) / np.sqrt(n)
        got = np.stack([g["xi"], g["eta"]], 1)
        got_se = np.stack([g["se_xi"], g["se_eta"]], 1)
        assert np.all(np.abs(got - mean) <= 1e-12 * np.maximum(np.abs(mean), 1e-3))
        assert np.all(np.abs(got_se - se) <= 1e-9 * se + 1e-18)
        steps = np.where(g["exit_step"] < 0, oracle_steps(t, dt), g["exit_step"]).sum(axis=1)
        assert np.array_equal(g["steps"], steps)
        only = fk.fk_interface_solve(wl.density, data, pts, t, dt, n, 5, steps=True)
        torch_cuda.cuda.synchronize()
        assert np.array_equal(only["steps"].cpu().numpy(), steps)
        assert "exit_step" not in only
        for k in ("xi", "eta", "se_xi", "se_eta"):
            assert np.array_equal(only[k].cpu().numpy(), g[k]), k


def test_device_nodes_and_mask(fk, torch_cuda, oracle_mod):
    """Node coordinates on the device and a device mask: a masked solve gives
    bitwise the full solve's results at its nodes (each node keeps its own
    random stream) and leaves the other nodes' outputs alone; a node outside
    the square or with a NaN coordinate gets NaN results without disturbing
    the others."""
    torch = torch_cuda
    wl = W.MOVING_BUMP_1521
    pts = wl.nodes()[::7]
    n, N = pts.shape[0], 700
    full = fk.fk_interface_solve(wl.density, wl.data, pts, 0.01, 1e-4, N, 3, 2, exit_step=True, scores=True,
                                 steps=True)
    dpts = torch.tensor(pts, device="cuda")
    again = fk.fk_interface_solve(wl.density, wl.data, dpts, 0.01, 1e-4, N, 3, 2, exit_step=True, scores=True,
                                  steps=True)
    rng = np.random.default_rng(11)
    mask = rng.random(n) < 0.3
    mask[0] = True
    sentinel = {k: torch.full_like(v, 7) for k, v in full.items() if not k.startswith("_") and k != "total_steps"}
    sentinel["total_steps"] = torch.zeros(1, dtype=torch.int64, device="cuda")
    print(f"[gpu] masked solve: {int(mask.sum())} of {n} nodes", flush=True)
    part = fk.fk_interface_solve(wl.density, wl.data, dpts, 0.01, 1e-4, N, 3, 2, exit_step=True, scores=True,
                                 steps=True, out=sentinel, mask=torch.tensor(mask.astype(np.uint8), device="cuda"))
    torch.cuda.synchronize()
    f = {k: v.cpu().numpy() for k, v in full.items() if not k.startswith("_")}
    for k in ("xi", "eta", "se_xi", "se_eta", "exit_step", "scores", "steps"):
        assert np.array_equal(again[k].cpu().numpy(), f[k]), k
        got = part[k].cpu().numpy()
        assert np.array_equal(got[mask], f[k][mask]), k
        assert np.all(got[~mask] == 7), k
    assert int(part["total_steps"][0]) == int(f["steps"][mask].sum())
    # bad nodes appended: NaN there, the others bitwise as before
    bad = np.vstack([pts, [[1.5, 0.5], [0.5, np.nan], [-1e-9, 0.2]]])
    g = run_gpu(fk, torch, wl.density, wl.data, bad, 0.01, 1e-4, N, 3, 2)
    for k in ("xi", "eta", "se_xi", "se_eta"):
        assert np.all(np.isnan(g[k][n:])), k
        assert np.array_equal(g[k][:n], f[k]), k
    assert np.array_equal(g["steps"][n:], [0, 0, 0])
    # the oracle on the masked nodes with their own ids
    idx = np.flatnonzero(mask)
    o = oracle_mod.fk_solve(wl.density, wl.data, pts[idx], 0.01, 1e-4, N, 3, 2, node_ids=idx, want_exit=True,
                            want_scores=True, threads=THREADS)
    assert_parity({k: v[mask] for k, v in f.items() if k != "total_steps"}, o, pts[idx])


def oracle_steps(t, dt):
    return int(math.ceil(t / dt - 1e-9))


def test_full_size_moving_bump_sampled(fk, torch_cuda, oracle_mod):
    """Full moving-bump workload (1521 nodes x 10^5 paths) in the benchmark's
    launch configuration; sampled paths recomputed one by one by the oracle,
    and four whole nodes recomputed in full."""
    wl = W.MOVING_BUMP_1521
    pts = wl.nodes()
    g = run_gpu(fk, torch_cuda, wl.density, wl.data, pts, wl.t, wl.dt, wl.n_paths)
    rng = np.random.default_rng(123)
    m = 256
    ni = rng.integers(0, len(pts), m)
    pi = rng.integers(0, wl.n_paths, m)
    sc, ex = oracle_mod.fk_paths(wl.density, wl.data, pts[ni], ni, pi, wl.t, wl.dt, wl.seed, threads=THREADS)
    ex_g = g["exit_step"][ni, pi]
    sc_g = g["scores"][ni, pi].astype(np.float64) + pts[ni].astype(np.float32).astype(np.float64)
    same = ex_g == ex
    print(f"sampled path exit match {same.mean():.4f}", flush=True)
    assert same.mean() >= 0.99
    assert np.all(np.abs(sc_g[same] - sc[same]) < 2e-5)
    # invariants over every node
    m_ = np.stack([g["xi"], g["eta"]], 1)
    s_ = np.stack([g["se_xi"], g["se_eta"]], 1)
    assert np.all(m_ >= -3 * s_) and np.all(m_ <= 1 + 3 * s_)
    assert int(g["total_steps"][0]) == int(g["steps"].sum())
    # four whole nodes, spread over the canonical order
    sel = np.array([0, 400, 800, 1500])
    o = oracle_mod.fk_solve(wl.density, wl.data, pts[sel], wl.t, wl.dt, wl.n_paths, wl.seed,
                            node_ids=sel, want_exit=True, want_scores=True, threads=THREADS)
    sub = {k: (g[k][sel] if k != "total_steps" else g[k]) for k in g}
    sub["total_steps"] = np.array([sub["steps"].sum()])
    assert_parity(sub, o, pts[sel])


@pytest.mark.parametrize("time_mode", [W.TIME_BACKWARD, W.TIME_FROZEN])
def test_paper_ring(fk, torch_cuda, oracle_mod, time_mode):
    """The paper's density w = 1/rho with the moving ring (Sect. 5), on the
    interface nodes of its 2 x 2 layout of a 41 x 41 grid; the drift jumps
    across the ring."""
    dens = W.paper_ring(time_mode, t_freeze=0.3)
    pts = W.interface_nodes(2, 2, 40)
    data = W.Data(t_init=0.25)
    g = run_gpu(fk, torch_cuda, dens, data, pts, 0.02, 5e-5, 2000, seed=21, level_id=3)
    o = run_oracle(oracle_mod, dens, data, pts, 0.02, 5e-5, 2000, seed=21, level_id=3)
    assert_parity(g, o, pts)
