"""Launch plans on the GPU: the autotuner (its choice is a valid plan, it
is cached, and every plan gives bitwise the same results -- node tiles
included), and the plan handle's graph capture: a captured solve replayed
between eager work, replayed on new node coordinates, re-captured for another
level (updated in place), and whole mesh steps run as graphs against the
same run taken eagerly."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _host(r):
    return {k: v.cpu().numpy() for k, v in r.items() if not k.startswith("_")}


def test_autotune_choice_is_cached_and_changes_nothing(fk):
    import torch
    wl = W.STATIC_BUMP_31
    pts = torch.tensor(wl.nodes(), device="cuda")
    p = fk.FkPlan()
    print("[gpu] autotune, 31 nodes x 1024 paths", flush=True)
    chosen = p.autotune(wl.density, wl.data, pts, wl.t, wl.dt, 1024)
    assert chosen["block"] in (64, 128, 256) and chosen["chunk"] in (32, 128, 512)
    assert chosen["node_tile"] in (1, 8) and chosen["blocks_per_cu"] >= 1
    again = fk.FkPlan().autotune(wl.density, wl.data, pts, wl.t, wl.dt, 1024)
    assert again == chosen                                      # the cache
    a = _host(fk.fk_interface_solve(wl.density, wl.data, pts, wl.t, wl.dt, 1024, 3, scores=True, steps=True,
                                    exit_step=True, plan=p))
    b = _host(fk.fk_interface_solve(wl.density, wl.data, pts, wl.t, wl.dt, 1024, 3, scores=True, steps=True,
                                    exit_step=True))
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    p.close()


@pytest.mark.parametrize("tile", [2, 4, 8, 64])
def test_node_tiles_change_only_the_schedule(fk, tile):
    import torch
    wl = W.MOVING_BUMP_1521
    pts = torch.tensor(wl.nodes()[::5], device="cuda")            # 305 nodes: partial last tiles
    ref = _host(fk.fk_interface_solve(wl.density, wl.data, pts, 0.01, 1e-4, 700, 2, scores=True, steps=True))
    got = _host(fk.fk_interface_solve(wl.density, wl.data, pts, 0.01, 1e-4, 700, 2, scores=True, steps=True,
                                      plan={"node_tile": tile, "chunk": 64}))
    for k in ref:
        assert np.array_equal(got[k], ref[k]), (tile, k)


def test_captured_solve_replays(fk):
    import torch
    wl = W.MOVING_BUMP_1521
    nodes = wl.nodes()
    n, N = 200, 512
    pts = torch.tensor(nodes[:n], device="cuda")
    out = {k: torch.empty(n, dtype=torch.float64, device="cuda") for k in ("xi", "eta", "se_xi", "se_eta")}
    out["total_steps"] = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(fk.fk_interface_workspace_bytes(n, N), dtype=torch.uint8, device="cuda")
    p = fk.FkPlan()
    s = torch.cuda.Stream()
    print("[gpu] capture of one interface solve", flush=True)
    with torch.cuda.stream(s):
        with p.capture():
            fk.fk_interface_solve(wl.density, wl.data, pts, 0.01, 1e-4, N, 4, 1, workspace=ws, out=out)
    ref = _host(fk.fk_interface_solve(wl.density, wl.data, pts, 0.01, 1e-4, N, 4, 1))
    keys = ("xi", "eta", "se_xi", "se_eta", "total_steps")
    for rep in range(3):
        for k in keys:
            out[k].fill_(-1)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            p.replay()
        s.synchronize()
        got = _host(out)
        for k in keys:
            assert np.array_equal(got[k], ref[k]), (rep, k)
        # eager work between replays
        fk.fk_interface_solve(wl.density, wl.data, torch.tensor(nodes[n:2 * n], device="cuda"), 0.01, 1e-4, 64, 9)
        torch.cuda.synchronize()
    # the graph reads the coordinates from the device: new contents, new solve
    pts.copy_(torch.tensor(nodes[500:500 + n], device="cuda"))
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        p.replay()
    s.synchronize()
    ref2 = _host(fk.fk_interface_solve(wl.density, wl.data, pts, 0.01, 1e-4, N, 4, 1))
    for k in ("xi", "eta", "se_xi", "se_eta"):
        assert np.array_equal(out[k].cpu().numpy(), ref2[k]), k
    # another level (other counters, another horizon): captured again, the
    # executable graph updated in place
    with torch.cuda.stream(s):
        with p.capture():
            fk.fk_interface_solve(wl.density, wl.data, pts, 0.012, 1e-4, N, 4, 2, workspace=ws, out=out)
        p.replay()
    s.synchronize()
    assert p.updates == 1
    ref3 = _host(fk.fk_interface_solve(wl.density, wl.data, pts, 0.012, 1e-4, N, 4, 2))
    for k in ("xi", "eta", "se_xi", "se_eta"):
        assert np.array_equal(out[k].cpu().numpy(), ref3[k]), k
    p.close()


@pytest.mark.parametrize("kw", [dict(cv_form="grid", key_points=True), dict(refit_every=0),
                                dict(cv_form="grid", density_data="grid")])
def test_mesh_steps_as_graphs(fk, kw):
    """Mesh steps recorded and replayed as graphs (each step's own time
    level and ping-pong buffers, the graph updated in place) give bitwise
    the run taken eagerly."""
    import torch
    from paper_1402_0266_amd.mesh_run import MeshRun, MeshRunConfig
    base = dict(px=4, m=16, dt_mesh=5e-4, substeps=20, n_steps=4, n_paths=1024, refit_every=0, cv_stride=2)
    base.update(kw)
    runs = []
    for graph in (False, True):
        print(f"[gpu] mesh run {kw} graph={graph}", flush=True)
        run = MeshRun(MeshRunConfig(**base, graph=graph))
        run.run()
        torch.cuda.synchronize()
        runs.append(run)
    e, g = runs
    assert g.plan.updates == base["n_steps"] - 1
    assert np.array_equal(e._iface.cpu().numpy(), g._iface.cpu().numpy())
    assert np.array_equal(e._quality.cpu().numpy(), g._quality.cpu().numpy())
    assert np.array_equal(e.xi.cpu().numpy(), g.xi.cpu().numpy()) and np.array_equal(e.eta.cpu().numpy(),
                                                                                    g.eta.cpu().numpy())
    if base.get("key_points"):
        assert e.n_keys == g.n_keys
