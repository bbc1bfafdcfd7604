"""TEST INFRASTRUCTURE -- the plain CPU oracle of the stochastic interface solver.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product (``paper_1402_0266_amd``)
never does, and this package never imports the product: the two share no code.

Contents:
  * ``fk_oracle.c``     -- FP64 Monte-Carlo oracle (Philox4x32-10, Box-Muller,
                           Euler-Maruyama, exit test, scoring, two-pass stats).
  * ``fd_reference.c``  -- FP64 finite-difference (ADI) solution of the PDE.
  * ``mlp.py``          -- FP64 NumPy oracle of the control-variate network.
  * ``subdomain.py``    -- FP64 SciPy oracle of the sub-domain implicit solve.

The C files are compiled with gcc into ``liboracle.so`` next to them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["fk_oracle.c", "fd_reference.c"]
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O3, OpenMP, no fast-math)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH):
        lib_m = os.path.getmtime(_LIB_PATH)
        if all(os.path.getmtime(s) <= lib_m for s in srcs):
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=c11", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.or_philox_batch.argtypes = [P, P, ctypes.c_int64, P]
        L.or_normals_batch.argtypes = [P, P, ctypes.c_int64, P]
        L.or_density_batch.argtypes = [ctypes.c_int, P, P, ctypes.c_int, ctypes.c_double, P, ctypes.c_int64, P, P]
        L.or_density_batch.restype = ctypes.c_int
        L.or_n_steps.argtypes = [ctypes.c_double, ctypes.c_double]
        L.or_n_steps.restype = ctypes.c_int64
        L.or_fk_solve.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  P, P, ctypes.c_int,
                                  P, P, ctypes.c_int64,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                  P, P, P, P, P]
        L.or_fk_solve.restype = ctypes.c_int
        L.or_fk_paths.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int,
                                  ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  P, P, ctypes.c_int,
                                  P, P, P, ctypes.c_int64,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                  ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, P, P]
        L.or_fk_paths.restype = ctypes.c_int
        L.or_mlp_eval.argtypes = [P, ctypes.c_double, P, ctypes.c_int64, P]
        L.or_mlp_eval.restype = ctypes.c_int
        L.or_fk_solve_cv.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     P, P, ctypes.c_int,
                                     P, P, ctypes.c_int64,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int64, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                                     ctypes.c_int, P, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                     P, P, P, P, P, P]
        L.or_fk_solve_cv.restype = ctypes.c_int
        L.or_fd_solve.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                  P, P, ctypes.c_int, P, P]
        L.or_fd_solve.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 words for counters ctr[n,4] and keys key[n,2] (uint32)."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    out = np.zeros_like(ctr)
    lib().or_philox_batch(_ptr(ctr), _ptr(key), ctr.shape[0], _ptr(out))
    return out


def normals(ra, rb) -> np.ndarray:
    """Box-Muller pairs [n,2] from the word pairs (ra, rb)."""
    ra = np.ascontiguousarray(ra, dtype=np.uint32).ravel()
    rb = np.ascontiguousarray(rb, dtype=np.uint32).ravel()
    out = np.zeros((ra.size, 2))
    lib().or_normals_batch(_ptr(ra), _ptr(rb), ra.size, _ptr(out))
    return out


def _wgrid(dens):
    """The nodal samples of a grid density (or None) and its cell count."""
    if dens.w_grid is None:
        return None, 0
    return np.ascontiguousarray(dens.w_grid, dtype=np.float64), dens.w_n


def density(dens, tau: float, pts):
    """(w[n], b[n,2]) of a ``workloads.Density`` at PDE time tau."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    par = dens.params()
    wg, wn = _wgrid(dens)
    w = np.zeros(pts.shape[0])
    b = np.zeros_like(pts)
    if lib().or_density_batch(dens.kind, _ptr(par), _ptr(wg), wn, tau, _ptr(pts), pts.shape[0], _ptr(w), _ptr(b)):
        raise ValueError("oracle rejected the density")
    return w, b


def sample_density(dens, tau: float, n: int) -> np.ndarray:
    """w of an analytic density at the nodes of an n-cell grid, [(n+1), (n+1)]
    indexed [j, i] with x = i/n, y = j/n."""
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x)
    w, _ = density(dens, tau, np.stack([X.ravel(), Y.ravel()], 1))
    return w.reshape(n + 1, n + 1)


def n_steps(t: float, dt: float) -> int:
    return int(lib().or_n_steps(t, dt))


def fk_solve(dens, data, pts, t, dt, n_paths, seed=0, level_id=0, stream=0,
             node_ids=None, want_exit=False, want_scores=False, threads=0):
    """Plain Monte-Carlo oracle.  Returns a dict with mean[n,2], se[n,2],
    steps[n] and optionally exit_step[n,N] (int32, -1 = survived) and
    scores[n,N,2]."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    n = pts.shape[0]
    par = dens.params()
    mean = np.zeros((n, 2))
    se = np.zeros((n, 2))
    steps = np.zeros(n, dtype=np.int64)
    ex = np.zeros((n, n_paths), dtype=np.int32) if want_exit else None
    sc = np.zeros((n, n_paths, 2)) if want_scores else None
    ids = None if node_ids is None else np.ascontiguousarray(node_ids, dtype=np.int64)
    gx = gy = None
    gn = 0
    if data.grid_xi is not None:
        gx = np.ascontiguousarray(data.grid_xi, dtype=np.float64)
        gy = np.ascontiguousarray(data.grid_eta, dtype=np.float64)
        gn = data.grid_n
    wg, wn = _wgrid(dens)
    rc = lib().or_fk_solve(dens.kind, dens.time_mode, _ptr(par), _ptr(wg), wn,
                           data.init_kind, data.bdry_kind, data.score_mode, data.t_init,
                           _ptr(gx), _ptr(gy), gn,
                           _ptr(pts), _ptr(ids), n,
                           t, dt, n_paths, seed, level_id, stream, threads,
                           _ptr(mean), _ptr(se), _ptr(ex), _ptr(sc), _ptr(steps))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    out = {"mean": mean, "se": se, "steps": steps}
    if want_exit:
        out["exit_step"] = ex
    if want_scores:
        out["scores"] = sc
    return out


def fk_paths(dens, data, pts, node_ids, path_ids, t, dt, seed=0, level_id=0, stream=0, threads=0):
    """Individual oracle paths: for each j, path path_ids[j] from pts[j] with
    Philox counter word 2 = node_ids[j].  Returns (scores[m,2], exit_step[m])."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    m = pts.shape[0]
    ids = np.ascontiguousarray(node_ids, dtype=np.int64).ravel()
    pids = np.ascontiguousarray(path_ids, dtype=np.int64).ravel()
    if ids.size != m or pids.size != m:
        raise ValueError("pts, node_ids and path_ids must have the same length")
    par = dens.params()
    sc = np.zeros((m, 2))
    ex = np.zeros(m, dtype=np.int32)
    gx = gy = None
    gn = 0
    if data.grid_xi is not None:
        gx = np.ascontiguousarray(data.grid_xi, dtype=np.float64)
        gy = np.ascontiguousarray(data.grid_eta, dtype=np.float64)
        gn = data.grid_n
    wg, wn = _wgrid(dens)
    rc = lib().or_fk_paths(dens.kind, dens.time_mode, _ptr(par), _ptr(wg), wn,
                           data.init_kind, data.bdry_kind, data.score_mode, data.t_init,
                           _ptr(gx), _ptr(gy), gn, _ptr(pts), _ptr(ids), _ptr(pids), m,
                           t, dt, seed, level_id, stream, threads, _ptr(sc), _ptr(ex))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return sc, ex


UHAT_MLP, UHAT_LINEAR, UHAT_SIN, UHAT_ZERO, UHAT_GRID, UHAT_MLP_BASE, UHAT_QUAD, UHAT_GRID_MLP = 0, 1, 2, 3, 4, 5, 6, 7
# GRID: the grid initial data; MLP_BASE: the identity map plus the MLP;
# QUAD: the test function (tau x^2, tau y^2); GRID_MLP: the grid initial data
# (bilinear) plus the MLP (martingale form: the mesh's gradient every 2 steps,
# the network's every `stride` steps)
CV_DYNKIN, CV_MARTINGALE = 0, 1   # forms of the control-variate estimator


def mlp_eval_c(flat, t_scale, txy) -> np.ndarray:
    """The C oracle's forward-mode MLP: [n, 2, 5] (value, dx, dy, dt, lap)."""
    flat = np.ascontiguousarray(flat, dtype=np.float64)
    txy = np.ascontiguousarray(txy, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((txy.shape[0], 2, 5))
    lib().or_mlp_eval(_ptr(flat), t_scale, _ptr(txy), txy.shape[0], _ptr(out))
    return out


def fk_solve_cv(dens, data, pts, t, dt, n_paths, seed=0, level_id=0, stream=0, node_ids=None,
                uhat=UHAT_MLP, flat=None, t_scale=0.1, stride=1, form=CV_DYNKIN, want_scores=False, want_exit=False,
                threads=0):
    """Control-variate oracle, Dynkin form (form=CV_DYNKIN) or martingale
    form (CV_MARTINGALE).  Returns dict: mean/se (CV), plain_mean/plain_se
    (same paths), optional cv_scores [n,N,2], exit_step."""
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    n = pts.shape[0]
    par = dens.params()
    out = {k: np.zeros((n, 2)) for k in ("mean", "se", "plain_mean", "plain_se")}
    cs = np.zeros((n, n_paths, 2)) if want_scores else None
    ex = np.zeros((n, n_paths), dtype=np.int32) if want_exit else None
    ids = None if node_ids is None else np.ascontiguousarray(node_ids, dtype=np.int64)
    fl = None if flat is None else np.ascontiguousarray(flat, dtype=np.float64)
    gx = gy = None
    gn = 0
    if data.grid_xi is not None:
        gx = np.ascontiguousarray(data.grid_xi, dtype=np.float64)
        gy = np.ascontiguousarray(data.grid_eta, dtype=np.float64)
        gn = data.grid_n
    wg, wn = _wgrid(dens)
    rc = lib().or_fk_solve_cv(dens.kind, dens.time_mode, _ptr(par), _ptr(wg), wn,
                              data.init_kind, data.bdry_kind, data.score_mode, data.t_init,
                              _ptr(gx), _ptr(gy), gn, _ptr(pts), _ptr(ids), n,
                              t, dt, n_paths, seed, level_id, stream, threads,
                              uhat, _ptr(fl), t_scale, stride, form,
                              _ptr(out["mean"]), _ptr(out["se"]), _ptr(out["plain_mean"]), _ptr(out["plain_se"]),
                              _ptr(cs), _ptr(ex))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    if want_scores:
        out["cv_scores"] = cs
    if want_exit:
        out["exit_step"] = ex
    return out


def fd_solve(dens, data, t, n, dtau, threads=0):
    """Finite-difference (ADI) solution; returns (xi, eta) as [(n+1), (n+1)]
    arrays indexed [j, i] with x = i/n, y = j/n."""
    if dens.w_grid is not None:
        raise ValueError("the FD reference takes analytic densities only")
    par = dens.params()
    xi = np.zeros((n + 1) * (n + 1))
    eta = np.zeros_like(xi)
    gx = gy = None
    if data.init_kind == 3:
        gx = np.ascontiguousarray(data.grid_xi, dtype=np.float64).ravel()
        gy = np.ascontiguousarray(data.grid_eta, dtype=np.float64).ravel()
    rc = lib().or_fd_solve(dens.kind, dens.time_mode, _ptr(par), data.init_kind, data.bdry_kind,
                           data.t_init, t, n, dtau, _ptr(gx), _ptr(gy), threads,
                           _ptr(xi), _ptr(eta))
    if rc != 0:
        raise ValueError("fd reference rejected its arguments")
    return xi.reshape(n + 1, n + 1), eta.reshape(n + 1, n + 1)


def sample_grid(grid, pts):
    """Values of a nodal grid at grid-aligned points (exact index lookup)."""
    n = grid.shape[0] - 1
    ij = np.rint(np.asarray(pts) * n).astype(np.int64)
    if np.max(np.abs(ij / n - pts)) > 1e-12:
        raise ValueError("points are not on the grid")
    return grid[ij[:, 1], ij[:, 0]]


def fd_reference_at(dens, data, t, pts, n_coarse=256, dtau=1e-5, threads=0):
    """Richardson-extrapolated FD values at grid-aligned points.

    Solves on n and 2n; returns (values[n_pts, 2], error_estimate[n_pts, 2]),
    the estimate being |u_2n - u_n| / 3 (second order in h)."""
    out = []
    for n in (n_coarse, 2 * n_coarse):
        xi, eta = fd_solve(dens, data, t, n, dtau, threads)
        out.append(np.stack([sample_grid(xi, pts), sample_grid(eta, pts)], axis=1))
    coarse, fine = out
    return fine + (fine - coarse) / 3.0, np.abs(fine - coarse) / 3.0
