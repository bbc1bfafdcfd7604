"""Pins of the sub-domain solve oracle and of the mesh-quality measures.

* w = 1, identity data: the linear maps are discrete steady states, kept to
  round-off by one backward-Euler step.
* w = 1, sine mode with zero boundary data: one step multiplies the mode by
  1 / (1 + D (8/h^2) sin^2(pi h / 2)) exactly (discrete eigenvalue).
* w = w(x): eta = y is kept exactly.
* Exact domain-decomposition identity: with interface values taken from the
  global solve, the sub-domain solves reproduce the global solution.
* Mesh quality: identity gives J = 1, skew = 0; an affine map gives its
  determinant and the angle between its rows.
* Equidistributed edges (Sect. 3): w = 1 gives the identity; w = w(x) gives
  xi = int_0^x w / int_0^1 w in closed form (erf) on the bottom and top
  edges and eta = y on the left and right ones.
"""
import math

import numpy as np
import pytest

import oracle.subdomain as S
import workloads as W


def grid(N):
    x = np.arange(N + 1) / N
    return np.meshgrid(x, x)


def test_identity_is_steady_for_w1():
    X, Y = grid(24)
    xi, eta = S.global_be_step(W.CONST, 0.0, 0.1, 24, X, Y)
    assert np.abs(xi - X).max() < 1e-13 and np.abs(eta - Y).max() < 1e-13


def test_sine_mode_discrete_eigenvalue():
    N, D = 32, 0.01
    X, Y = grid(N)
    phi = np.sin(math.pi * X) * np.sin(math.pi * Y)
    xi, eta = S.global_be_step(W.CONST, 0.0, D, N, phi, phi, bdry="zero")
    h = 1.0 / N
    factor = 1.0 / (1.0 + D * 8.0 / h ** 2 * math.sin(math.pi * h / 2) ** 2)
    assert np.abs(xi - factor * phi).max() < 1e-13 and np.array_equal(xi, eta)


def test_ridge_keeps_eta_linear():
    X, Y = grid(24)
    xi, eta = S.global_be_step(W.ridge(), 0.0, 0.05, 24, X, Y)
    assert np.abs(eta - Y).max() < 1e-13
    assert np.abs(xi - X).max() > 1e-3


@pytest.mark.parametrize("px,m,dens", [(4, 8, W.moving_bump()), (3, 10, W.static_bump()),
                                       (2, 16, W.two_bumps(W.TIME_FROZEN, 0.03))])
def test_exact_domain_decomposition_identity(px, m, dens):
    N = px * m
    X, Y = grid(N)
    # a non-trivial previous mesh
    xi0 = X + 0.02 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    eta0 = Y + 0.015 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    gxi, geta = S.global_be_step(dens, 0.04, 0.02, N, xi0, eta0)
    ij = S.interface_index(px, m)
    sxi, seta = S.subdomain_be_step(dens, 0.04, 0.02, px, m, xi0, eta0, gxi[ij[:, 1], ij[:, 0]],
                                    geta[ij[:, 1], ij[:, 0]])
    assert np.abs(sxi - gxi).max() < 1e-12 and np.abs(seta - geta).max() < 1e-12
    # and the step moved the mesh
    assert np.abs(gxi - xi0).max() > 1e-4


@pytest.mark.parametrize("px,py,N,dens", [(2, 3, 24, W.moving_bump()), (4, 1, 24, W.static_bump()),
                                          (1, 3, 18, W.two_bumps(W.TIME_FROZEN, 0.03)),
                                          (3, 2, 30, W.paper_ring(W.TIME_FROZEN, 0.1))])
def test_exact_domain_decomposition_identity_rect(px, py, N, dens):
    """The same identity for px x py splits (sub-domains wider than tall and
    taller than wide, a single row or column of them)."""
    X, Y = grid(N)
    xi0 = X + 0.02 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    eta0 = Y + 0.015 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    gxi, geta = S.global_be_step(dens, 0.04, 0.02, N, xi0, eta0)
    ij = S.interface_index_rect(px, py, N)
    assert len(ij) == (px - 1) * (N - 1) + (py - 1) * (N - px)
    sxi, seta = S.subdomain_be_step_rect(dens, 0.04, 0.02, px, py, N, xi0, eta0, gxi[ij[:, 1], ij[:, 0]],
                                         geta[ij[:, 1], ij[:, 0]])
    assert np.abs(sxi - gxi).max() < 1e-12 and np.abs(seta - geta).max() < 1e-12
    assert np.abs(gxi - xi0).max() > 1e-4


def test_interface_index_matches_canonical_nodes():
    for px, m in ((2, 16), (4, 64), (8, 96)):
        ij = S.interface_index(px, m)
        pts = W.interface_nodes(px, px, px * m)
        assert np.array_equal(ij / (px * m), pts)
    for px, py, N in ((2, 4, 128), (8, 3, 96), (5, 7, 140)):
        ij = S.interface_index_rect(px, py, N)
        assert np.array_equal(ij / N, W.interface_nodes(px, py, N))


def test_mesh_quality_closed_forms():
    X, Y = grid(16)
    assert S.mesh_quality(X, Y) == pytest.approx((1.0, 0.0), abs=1e-12)
    a, b, c, d = 1.2, 0.3, -0.1, 0.8
    jac, skew = S.mesh_quality(a * X + b * Y, c * X + d * Y)
    assert jac == pytest.approx(a * d - b * c, abs=1e-12)
    assert skew == pytest.approx(abs(a * c + b * d) / (math.hypot(a, b) * math.hypot(c, d)), abs=1e-12)


def test_equidistributed_edges_closed_forms():
    N = 16
    gx, gy = S.boundary_grid(N, "equidistributed", W.CONST, 0.0)
    ix, iy = S.boundary_grid(N, "identity")
    edge = np.zeros((N + 1, N + 1), dtype=bool)
    edge[0, :] = edge[-1, :] = edge[:, 0] = edge[:, -1] = True
    assert np.abs(gx - ix)[edge].max() < 1e-13 and np.abs(gy - iy)[edge].max() < 1e-13
    A, s2, c = 10.0, 0.01, 0.35
    dens = W.ridge(A, s2, c)
    gx, gy = S.boundary_grid(N, "equidistributed", dens, 0.0)
    x = np.arange(N + 1) / N
    F = lambda u: u + A * math.sqrt(math.pi * s2) / 2 * (math.erf((u - c) / math.sqrt(s2)) + math.erf(c / math.sqrt(s2)))  # noqa: E731
    exact = np.array([F(u) / F(1.0) for u in x])
    assert np.abs(gx[0, :] - exact).max() < 1e-12 and np.abs(gx[-1, :] - exact).max() < 1e-12
    assert np.abs(gy[:, 0] - x).max() < 1e-12 and np.abs(gy[:, -1] - x).max() < 1e-12
    assert np.all(gx[:, 0] == 0.0) and np.all(gx[:, -1] == 1.0)
    assert np.all(gy[0, :] == 0.0) and np.all(gy[-1, :] == 1.0)
