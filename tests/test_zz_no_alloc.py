"""The interface solve without a workspace (fk_interface_solve_noalloc):
its tables and sums live in the library's static device scratch.  Called
through the C ABI, it gives bitwise the results of fk_interface_solve on the
same inputs, on two calls in a row (the second smaller, so stale scratch
contents would show)."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _outputs(torch, n, n_paths):
    o = {k: torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
         for k in ("xi", "eta", "se_xi", "se_eta")}
    o["exit_step"] = torch.full((n, n_paths), -7, dtype=torch.int32, device="cuda")
    o["scores"] = torch.zeros((n, n_paths, 2), dtype=torch.float32, device="cuda")
    o["steps"] = torch.zeros(n, dtype=torch.int64, device="cuda")
    o["total_steps"] = torch.zeros(1, dtype=torch.int64, device="cuda")
    return o


def _call_noalloc(fk, torch, dens, data, pts, t, dt, n_paths, seed, level_id, o):
    pts = torch.as_tensor(np.ascontiguousarray(pts, dtype=np.float64), device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fk.library().fk_interface_solve_noalloc(
        ctypes.byref(fk._density(dens)), ctypes.byref(fk._data(data)), pts.data_ptr(), None,
        pts.shape[0], t, dt, n_paths, seed, level_id, o["xi"].data_ptr(), o["eta"].data_ptr(),
        o["se_xi"].data_ptr(), o["se_eta"].data_ptr(), o["exit_step"].data_ptr(), o["scores"].data_ptr(),
        o["steps"].data_ptr(), o["total_steps"].data_ptr(), None, stream)
    assert rc == 0, fk.fk_last_error()
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in o.items()}


def test_noalloc_matches_the_workspace_solve(fk):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    cases = [
        (W.MOVING_BUMP_1521.density, W.Data(), W.MOVING_BUMP_1521.nodes()[::3], 0.02, 1e-5, 3000, 4, 1),
        (W.static_bump(), W.Data(), W.STATIC_BUMP_31.nodes()[:9], 0.05, 1e-4, 700, 9, 2),
    ]
    for dens, data, pts, t, dt, n, seed, lid in cases:
        print(f"[gpu] noalloc: nodes={len(pts)} N={n} t={t} dt={dt} seed={seed}", flush=True)
        got = _call_noalloc(fk, torch, dens, data, pts, t, dt, n, seed, lid, _outputs(torch, len(pts), n))
        ref = fk.fk_interface_solve(dens, data, pts, t, dt, n, seed, lid, exit_step=True, scores=True, steps=True)
        torch.cuda.synchronize()
        for k in ("xi", "eta", "se_xi", "se_eta", "exit_step", "scores", "steps", "total_steps"):
            assert np.array_equal(got[k], ref[k].cpu().numpy()), k
        assert np.all(np.isfinite(got["xi"])) and np.all(got["se_xi"] > 0)
