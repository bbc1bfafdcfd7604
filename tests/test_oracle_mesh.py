"""Pins of the mesh-step oracle: grid initial data, the frozen density, and
the composition of the interface solve with the sub-domain solves.

* Grid data holding the transposed identity (xi grid = y, eta grid = x) is
  interpolated exactly, so with no exits the xi estimate equals the eta
  estimate of identity data on the same paths (grid orientation and the
  [j][i] layout).
* Grid data sampling phi = sin(pi x) sin(pi y) on an n-cell grid differs from
  phi by at most the bilinear interpolation bound (h^2/8)(|phi_xx| + |phi_yy|)
  = pi^2 h^2 / 4 per path; exits score the same boundary data (cell lookup
  and weights).
* A moving bump frozen at t_f is the static bump centred at c(t_f) (the
  frozen time argument).
* w = 1: a domain-decomposition step of a perturbed mesh agrees with the
  global backward-Euler step at the interface nodes within the Monte-Carlo
  error, and the sub-domain solves spread no more than the interface
  discrepancy into the interiors (discrete maximum principle).
* Two counter-rotating bumps, frozen: the interface estimates follow the
  global solution of the same flow (finely time-stepped), and over a few
  mesh steps the decomposed mesh keeps the quality of the global
  backward-Euler step from the same mesh.
"""
import math
import os

import numpy as np

import oracle.mesh_step as MS
import oracle.subdomain as S
import workloads as W

THREADS = min(8, os.cpu_count() or 1)


def nodal(N):
    x = np.arange(N + 1) / N
    return np.meshgrid(x, x)


def test_grid_transposed_identity_is_exact(oracle_mod):
    X, Y = nodal(64)
    dens = W.moving_bump(W.TIME_FROZEN, 0.02)
    pts = W.uniform_points(12, seed=3, lo=0.42, hi=0.58)
    t, dt, N = 1e-3, 1e-4, 400
    ident = oracle_mod.fk_solve(dens, W.Data(), pts, t, dt, N, seed=5, want_exit=True, want_scores=True,
                                threads=THREADS)
    grid = oracle_mod.fk_solve(dens, W.Data(init_kind=W.DATA_GRID, grid_xi=Y, grid_eta=X), pts, t, dt, N, seed=5,
                               want_exit=True, want_scores=True, threads=THREADS)
    assert np.all(ident["exit_step"] == -1) and np.all(grid["exit_step"] == -1)
    assert np.abs(grid["scores"][:, :, 0] - ident["scores"][:, :, 1]).max() < 1e-14
    assert np.abs(grid["scores"][:, :, 1] - ident["scores"][:, :, 0]).max() < 1e-14


def test_grid_sine_mode_within_interpolation_bound(oracle_mod):
    n = 128
    X, Y = nodal(n)
    phi = np.sin(math.pi * X) * np.sin(math.pi * Y)
    dens = W.static_bump()
    pts = W.uniform_points(16, seed=4)
    t, dt, N = 0.02, 1e-3, 300
    exact = oracle_mod.fk_solve(dens, W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_SIN), pts, t, dt, N, seed=2,
                                want_exit=True, want_scores=True, threads=THREADS)
    grid = oracle_mod.fk_solve(dens, W.Data(init_kind=W.DATA_GRID, bdry_kind=W.DATA_SIN, grid_xi=phi, grid_eta=phi),
                               pts, t, dt, N, seed=2, want_exit=True, want_scores=True, threads=THREADS)
    assert np.array_equal(exact["exit_step"], grid["exit_step"])
    d = np.abs(grid["scores"] - exact["scores"])
    bound = math.pi ** 2 / (4 * n * n)
    exited = exact["exit_step"] >= 0
    assert np.all(d[exited] == 0.0)
    assert d.max() <= bound * (1 + 1e-9)
    assert d[~exited].max() > 0.05 * bound       # the interpolant is really used


def test_frozen_moving_bump_is_static_bump_at_its_centre(oracle_mod):
    tf = 0.037
    mov = W.moving_bump(W.TIME_FROZEN, tf)
    c = (0.5 + 0.25 * math.cos(2 * math.pi * tf), 0.5 + 0.25 * math.sin(2 * math.pi * tf))
    sta = W.Density(W.KIND_BUMP, W.TIME_BACKWARD, amp=20.0, width2=0.005, cx=c[0], cy=c[1])
    pts = W.interface_nodes(4, 4, 16)
    t, dt, N = 0.01, 1e-4, 500
    a = oracle_mod.fk_solve(mov, W.Data(), pts, t, dt, N, seed=8, want_exit=True, threads=THREADS)
    b = oracle_mod.fk_solve(sta, W.Data(), pts, t, dt, N, seed=8, want_exit=True, threads=THREADS)
    assert np.mean(a["exit_step"] == b["exit_step"]) >= 0.999
    same = np.all(a["exit_step"] == b["exit_step"], axis=1)
    assert same.sum() >= len(pts) - 1
    assert np.abs(a["mean"][same] - b["mean"][same]).max() < 1e-9


def test_dd_step_heat_equation_matches_global_step(oracle_mod):
    px, m = 4, 8
    N = px * m
    X, Y = nodal(N)
    xi0 = X + 0.02 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    eta0 = Y + 0.015 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    D, n_paths = 5e-4, 20000
    xi, eta, mc = MS.dd_step(W.CONST, 0.0, D, 20, px, m, xi0, eta0, n_paths, seed=1, threads=THREADS)
    gxi, geta = S.global_be_step(W.CONST, 0.0, D, N, xi0, eta0)
    ij = S.interface_index(px, m)
    g_if = np.stack([gxi[ij[:, 1], ij[:, 0]], geta[ij[:, 1], ij[:, 0]]], 1)
    # Backward Euler against the exact flow over D for the two modes
    # (lambda = 5 pi^2): |exp(-D lambda) - 1 / (1 + D lambda)| 0.02 < 1e-5;
    # the 5-point Laplacian's eigenvalue error adds ~1e-5.  4.5 standard
    # errors: the largest of 354 normal deviates exceeds it with p ~ 0.2%.
    d = np.abs(mc["mean"] - g_if)
    assert np.all(d <= 4.5 * mc["se"] + 2e-5), (d / mc["se"]).max()
    z = (mc["mean"] - g_if) / mc["se"]
    assert abs(z.mean()) < 4 / math.sqrt(z.size) + 0.05 and 0.7 < z.std() < 1.3
    # the sub-domain solves: interiors within the interface discrepancy
    assert np.abs(xi - gxi).max() <= np.abs(mc["mean"][:, 0] - g_if[:, 0]).max() + 1e-12
    assert np.abs(eta - geta).max() <= np.abs(mc["mean"][:, 1] - g_if[:, 1]).max() + 1e-12


def test_two_bump_interface_values_follow_the_frozen_flow(oracle_mod):
    """From the identity mesh the frozen two-bump flow has a stiff initial
    layer, so one backward-Euler step of dt_mesh differs from the exact flow
    by several standard errors; forty sub-steps bring the global solve to
    the flow the Monte-Carlo estimates, within their error (ten leave a
    time-discretisation error of about one standard error at the worst
    nodes: max |z| 4.6 there against 3.4 with forty, on the same paths)."""
    px, m, D = 4, 8, 5e-4
    N = px * m
    xi0, eta0 = nodal(N)
    dens = W.two_bumps(W.TIME_FROZEN, 0.0)
    mc = MS.interface_solve(dens, 0.0, D, 20, px, m, xi0, eta0, 40000, threads=THREADS)
    a, b = xi0, eta0
    for _ in range(40):
        a, b = S.global_be_step(dens, 0.0, D / 40, N, a, b)
    ij = S.interface_index(px, m)
    z = (mc["mean"] - np.stack([a[ij[:, 1], ij[:, 0]], b[ij[:, 1], ij[:, 0]]], 1)) / mc["se"]
    assert np.abs(z).max() < 4.5 and 0.8 < z.std() < 1.25, (np.abs(z).max(), z.std())


def test_two_bump_dd_keeps_global_quality(oracle_mod):
    """The decomposed mesh keeps the quality of the global step.  The
    interface noise moves the Jacobian of the cells beside an interface by
    about 2 SE / h, so the paths per node are chosen to keep that near 1%."""
    px, m, D = 4, 8, 5e-4
    N = px * m
    xi, eta = nodal(N)
    for n in range(3):
        tn = n * D
        dens = W.two_bumps(W.TIME_FROZEN, tn)
        gxi, geta = S.global_be_step(dens, tn, D, N, xi, eta)
        xi, eta, _ = MS.dd_step(dens, tn, D, 20, px, m, xi, eta, 40000, seed=0, level_id=n, threads=THREADS)
        jg, sg = S.mesh_quality(gxi, geta)
        jd, sd = S.mesh_quality(xi, eta)
        assert jd > 0 and abs(jd - jg) <= 0.05 * jg and abs(sd - sg) <= 0.02, (n, jd, jg, sd, sg)
        assert jg < 0.95                         # the bumps really deform the mesh


def test_exit_scoring_near_a_compressed_boundary(oracle_mod):
    """w = 1 and a mesh whose normal slope at x = 0 is 1/2 (xi = x (1 + x) / 2).
    The discrete exit test sees a path one step's overshoot past the edge.
    The identity continued unclamped has slope 1 there, and a projected exit
    point drops the overshoot: both bias the nodes next to the edge.  The
    mesh continued bilinearly (its edge nodes hold the identity data) has the
    solution's slope and is unbiased to first order; so is the Brownian-bridge
    test, which finds the crossings within a step and scores the mesh's edge
    at them.  Reference: the global solve over the mesh step in 10
    backward-Euler sub-steps."""
    px, m, D = 4, 16, 5e-4
    N = px * m
    X, Y = nodal(N)
    xi0, eta0 = X * (1 + X) / 2, Y.copy()
    a, b = xi0, eta0
    for _ in range(10):
        a, b = S.global_be_step(W.CONST, 0.0, D / 10, N, a, b)
    ij_all = S.interface_index(px, m)
    ids = np.array([k for k, (i, j) in enumerate(ij_all) if i in (1, 2) and j == 2 * m])
    ij = ij_all[ids]
    ref = a[ij[:, 1], ij[:, 0]]
    z = {}
    for mode in (W.SCORE_UNCLAMPED, W.SCORE_PROJECT, W.SCORE_EXTEND, W.SCORE_BRIDGE):
        mc = MS.interface_solve(W.CONST, 0.0, D, 20, px, m, xi0, eta0, 200000, node_ids=ids, score_mode=mode,
                                bdry_kind=W.DATA_GRID if mode == W.SCORE_BRIDGE else W.DATA_IDENTITY,
                                threads=THREADS)
        z[mode] = (mc["mean"][:, 0] - ref) / mc["se"][:, 0]
    assert np.all(np.abs(z[W.SCORE_EXTEND]) < 4), z
    assert np.all(np.abs(z[W.SCORE_BRIDGE]) < 4), z
    assert z[W.SCORE_UNCLAMPED][0] < -8 and z[W.SCORE_PROJECT][0] > 8, z
