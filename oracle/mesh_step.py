"""TEST INFRASTRUCTURE -- FP64 oracle of one stochastic domain-decomposition
mesh step (Sect. 4), composed of the pinned pieces in the paper's order:

1. the density is frozen at t^n;
2. the interface values at t^{n+1} = t^n + dt_mesh are Feynman-Kac Monte-Carlo
   estimates (Sect. 3) with the mesh at t^n as initial data, bilinear in the
   nodal grid, and the identity map as boundary data, an exit scored with
   the mesh continued past the edge (its edge nodes hold the identity data)
   -- plain (fk_solve) or, given a network, a control-variate form
   (fk_solve_cv);
3. each sub-domain takes one backward-Euler step with those interface values
   as Dirichlet data (subdomain_be_step).

Only tests, the package's smoke check and the benchmark's CPU baseline use it.
"""
from __future__ import annotations

import numpy as np

import oracle as _oracle
import oracle.keypoints as _keys
import oracle.subdomain as _sub

DATA_IDENTITY = 0
DATA_GRID = 3
SCORE_EXTEND = 2      # exits: the grid continued bilinearly past the edge
UHAT_MLP = 1


class _GridData:
    """The fields the oracle's solvers read for grid initial data."""

    def __init__(self, t_init, xi, eta, score_mode, bdry_kind=DATA_IDENTITY):
        self.init_kind = DATA_GRID
        self.bdry_kind = bdry_kind
        self.score_mode = score_mode
        self.t_init = float(t_init)
        self.grid_xi = np.ascontiguousarray(xi, dtype=np.float64)
        self.grid_eta = np.ascontiguousarray(eta, dtype=np.float64)
        self.grid_n = self.grid_xi.shape[0] - 1


def interface_points(px: int, m: int) -> np.ndarray:
    """Coordinates of the interface nodes in the sub-domain solve's order."""
    ij = _sub.interface_index(px, m)
    return ij.astype(np.float64) / (px * m)


def interface_solve(dens, tn, dt_mesh, substeps, px, m, xi_n, eta_n, n_paths, seed=0, level_id=0,
                    node_ids=None, flat=None, t_scale=0.1, stride=10, form=0, score_mode=SCORE_EXTEND,
                    bdry_kind=DATA_IDENTITY, threads=0):
    """Step 2: interface estimates (dict with mean [n, 2], se [n, 2]) at the
    nodes node_ids (default all) of px x px sub-domains.  Exits score the
    mesh continued bilinearly past the edge by default (score_mode); with a
    projecting score mode, bdry_kind DATA_GRID scores the mesh itself at the
    projected exit point."""
    pts = interface_points(px, m)
    if node_ids is not None:
        # the nodes keep their indices in the full set: those key the paths' counters
        node_ids = np.asarray(node_ids, dtype=np.int64)
        pts = pts[node_ids]
    data = _GridData(tn, xi_n, eta_n, score_mode, bdry_kind)
    dt = dt_mesh / substeps
    if flat is None:
        return _oracle.fk_solve(dens, data, pts, dt_mesh, dt, n_paths, seed=seed, level_id=level_id,
                                node_ids=node_ids, threads=threads)
    return _oracle.fk_solve_cv(dens, data, pts, dt_mesh, dt, n_paths, seed=seed, level_id=level_id,
                               node_ids=node_ids, uhat=UHAT_MLP, flat=flat, t_scale=t_scale, stride=stride,
                               form=form, threads=threads)


def dd_step(dens, tn, dt_mesh, substeps, px, m, xi_n, eta_n, n_paths, seed=0, level_id=0,
            score_mode=SCORE_EXTEND, threads=0):
    """One plain mesh step: returns (xi, eta, interface estimates)."""
    mc = interface_solve(dens, tn, dt_mesh, substeps, px, m, xi_n, eta_n, n_paths, seed=seed,
                         level_id=level_id, score_mode=score_mode, threads=threads)
    xi, eta = _sub.subdomain_be_step(dens, tn, dt_mesh, px, m, xi_n, eta_n, mc["mean"][:, 0], mc["mean"][:, 1])
    return xi, eta, mc


def dd_step_keys(dens, tn, dt_mesh, substeps, px, m, xi_n, eta_n, n_paths, w_grid, tol=1e-2, max_gap=None,
                 bdry="identity", seed=0, level_id=0, score_mode=SCORE_EXTEND, threads=0):
    """One plain mesh step with key points (Sect. 4 speed-up): the Monte-Carlo
    solve at the key points chosen from w_grid (the density's samples at t^n
    on the mesh grid), their paths keyed by their position in the key list;
    the other interface nodes by the interpolant along their line through the
    boundary data at its ends; then the sub-domain solves.  Returns (xi, eta,
    key estimates, key mask)."""
    mask, pts = _keys.key_points(w_grid, px, m, tol, max_gap)
    data = _GridData(tn, xi_n, eta_n, score_mode)
    mc = _oracle.fk_solve(dens, data, pts, dt_mesh, dt_mesh / substeps, n_paths, seed=seed, level_id=level_id,
                          threads=threads)
    gx, gy = _sub.boundary_grid(px * m, bdry, dens, tn)
    iface = _keys.interpolate_interface(px, m, mask, mc["mean"], gx, gy)
    xi, eta = _sub.subdomain_be_step(dens, tn, dt_mesh, px, m, xi_n, eta_n, iface[:, 0], iface[:, 1], bdry=bdry)
    return xi, eta, mc, mask


SCORE_BRIDGE = 3
DATA_GRID_BOUNDARY = 3   # boundary data read from the grid at the projected exit point


def steady_start(px, m, bdry, dens):
    """The grid a steady solve starts from: the identity map with the outer
    boundary data on its edge nodes."""
    N = px * m
    x = np.arange(N + 1) / N
    X, Y = np.meshgrid(x, x)
    gx, gy = _sub.boundary_grid(N, bdry, dens, 0.0)
    edge = np.zeros((N + 1, N + 1), dtype=bool)
    edge[0, :] = edge[-1, :] = edge[:, 0] = edge[:, -1] = True
    return np.where(edge, gx, X), np.where(edge, gy, Y)


def steady_dd(dens, px, m, n_paths, dt, horizon, bdry="identity", seed=0, threads=0):
    """The elliptic (steady) stochastic domain decomposition (eq. (2)): paths
    run until they leave the square (Brownian-bridge exit test, the grid's
    edge nodes as boundary data; the horizon only caps the rare long path,
    which then scores the start grid), then each sub-domain solves the
    steady system with the interface values as Dirichlet data.  The density
    is static (frozen).  Returns (xi, eta, interface estimates)."""
    sx, sy = steady_start(px, m, bdry, dens)
    data = _GridData(0.0, sx, sy, SCORE_BRIDGE, bdry_kind=DATA_GRID_BOUNDARY)
    mc = _oracle.fk_solve(dens, data, interface_points(px, m), horizon, dt, n_paths, seed=seed, want_exit=True,
                          threads=threads)
    xi, eta = _sub.subdomain_be_step(dens, 0.0, np.inf, px, m, sx, sy, mc["mean"][:, 0], mc["mean"][:, 1],
                                     bdry=bdry)
    return xi, eta, mc
