"""Shared parity check of a GPU interface solve against the oracle.

The contract, per node and component, on the same Philox counters:
  * exit steps identical on >= 99.9% of all paths;
  * mean within 3 standard errors of the oracle's, and within 1e-5 absolute;
  * standard error within 1% relative.
A path whose exit step differs (its position sat within rounding of the
boundary at some step) contributes a different score to the mean; the
99.9% clause allows such paths, so for a node that has any, the 1e-5 bound
is applied to the means over the paths whose exit steps agree, and the whole
mean must stay within 3 standard errors plus the mismatched paths' share.
"""
import numpy as np


def gpu_scores_abs(g, pts, shifted: bool):
    """GPU per-path scores as absolute values (FP64)."""
    sc = g["scores"].astype(np.float64)
    if shifted:
        sc = sc + pts.astype(np.float32).astype(np.float64)[:, None, :]
    return sc


def assert_parity(g, o, pts=None, shifted=True, abs_tol=1e-5, match_min=0.999, label="", exact_steps=True):
    ex_g, ex_o = g["exit_step"], o["exit_step"]
    same = ex_g == ex_o
    match = float(np.mean(same))
    mean_g = np.stack([g["xi"], g["eta"]], axis=1)
    se_g = np.stack([g["se_xi"], g["se_eta"]], axis=1)
    d = np.abs(mean_g - o["mean"])
    n_paths = ex_g.shape[1]
    bad = np.where(~np.all(same, axis=1))[0]
    print(f"{label} exit-step match {match:.6f} ({int((~same).sum())} paths on {len(bad)} nodes); "
          f"max |mean diff| {d.max():.3e}; max diff/se {np.max(d / np.maximum(o['se'], 1e-300)):.3f}", flush=True)
    assert match >= match_min
    ok = np.ones(len(d), dtype=bool)
    ok[bad] = False
    assert np.all(d[ok] <= abs_tol)
    assert np.all(d[ok] <= 3.0 * o["se"][ok] + 1e-15)
    if len(bad):
        assert "scores" in g and "scores" in o, "node with mismatched paths: per-path scores needed"
        sg = gpu_scores_abs(g, pts, shifted)
        so = o["scores"]
        for i in bad:
            m = same[i]
            dm = np.abs(sg[i, m].mean(axis=0) - so[i, m].mean(axis=0))
            k = int((~m).sum())
            assert np.all(dm <= abs_tol), (i, dm)
            assert np.all(d[i] <= 3.0 * o["se"][i] + 2.0 * k / n_paths), (i, d[i])
    nz = o["se"] > 0
    assert np.all(np.abs(se_g[nz] - o["se"][nz]) <= 0.01 * o["se"][nz])
    if exact_steps and "steps" in g and match == 1.0:
        assert np.array_equal(g["steps"], o["steps"])
    if "steps" in g and "total_steps" in g:
        assert int(g["total_steps"][0]) == int(g["steps"].sum())
