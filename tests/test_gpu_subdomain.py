"""GPU sub-domain solves and mesh quality against the FP64 SciPy oracle."""
import math

import numpy as np
import pytest

import oracle.subdomain as S
import workloads as W

pytestmark = pytest.mark.gpu


def grid(N):
    x = np.arange(N + 1) / N
    return np.meshgrid(x, x)


def prev_mesh(N):
    X, Y = grid(N)
    return (X + 0.02 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y),
            Y + 0.015 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y))


def cuda(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("px,m,dens,t_w,D", [
    (4, 8, W.moving_bump(), 0.04, 0.02),
    (3, 10, W.static_bump(), 0.0, 0.05),
    (2, 32, W.two_bumps(W.TIME_FROZEN, 0.03), 0.03, 5e-4),
    (1, 20, W.ridge(), 0.0, 0.01),
    (4, 64, W.moving_bump(), 0.0, 0.1),          # 4x4 layout on 64x64 grids
    (8, 96, W.two_bumps(W.TIME_FROZEN, 0.05), 0.05, 5e-4),  # 8x8 layout on 96x96 grids
    # every side of the one-wavefront eliminations: 12 (whole system), 16
    # and 24 (both ends, separator); 48 and 40 on the tile kernel (40: a
    # window narrower than its 48 lanes)
    (3, 12, W.moving_bump(), 0.07, 0.01),
    (2, 16, W.paper_ring(W.TIME_FROZEN, 0.6), 0.6, 1e-3),
    (3, 24, W.two_bumps(W.TIME_FROZEN, 0.01), 0.01, 2e-3),
    (2, 48, W.static_bump(), 0.0, 1e-3),
    (2, 40, W.ridge(), 0.0, 0.02),
])
def test_subdomain_against_oracle(fk, px, m, dens, t_w, D):
    import torch
    N = px * m
    xi0, eta0 = prev_mesh(N)
    rng = np.random.default_rng(px * 1000 + m)
    ij = S.interface_index(px, m)
    # interface data: the previous mesh plus a small perturbation
    ix = xi0[ij[:, 1], ij[:, 0]] + 1e-3 * rng.standard_normal(len(ij))
    iy = eta0[ij[:, 1], ij[:, 0]] + 1e-3 * rng.standard_normal(len(ij))
    print(f"[gpu] subdomain px={px} m={m} kind={dens.kind}", flush=True)
    gx, gy = fk.subdomain_solve(dens, t_w, D, px, m, cuda(xi0), cuda(eta0), cuda(ix), cuda(iy))
    torch.cuda.synchronize()
    ox, oy = S.subdomain_be_step(dens, t_w, D, px, m, xi0, eta0, ix, iy)
    err = max(np.abs(gx.cpu().numpy() - ox).max(), np.abs(gy.cpu().numpy() - oy).max())
    print(f"max |gpu - oracle| = {err:.3e}", flush=True)
    assert err < 1e-12


@pytest.mark.parametrize("px,py,N,dens,t_w,D", [
    (2, 3, 48, W.moving_bump(), 0.04, 0.02),             # 24 x 16 cells: y is the fast index, 16-wide window
    (4, 1, 64, W.static_bump(), 0.0, 0.05),              # 16 x 64: x fast, one row of sub-domains
    (1, 2, 96, W.two_bumps(W.TIME_FROZEN, 0.03), 0.03, 5e-4),   # 96 x 48: tile kernel, 48-wide window
    (3, 2, 150, W.moving_bump(), 0.02, 0.01),            # 50 x 75: window 50 in a 64-lane-row tile
    (8, 6, 768, W.two_bumps(W.TIME_FROZEN, 0.05), 0.05, 5e-4),  # 96 x 128: the 768-cell grid, 48 sub-domains
    (1, 1, 120, W.ridge(), 0.0, 0.02),                   # one 120 x 120 domain: the widest window
    (3, 5, 30, W.static_bump(), 0.0, 0.05),              # 10 x 6: one end, no separator
    # 2 x 8 cells: one unknown across, a column of 7 (the fast and slow neighbours share a band offset)
    (4, 1, 8, W.Density(W.KIND_BUMP, W.TIME_FROZEN, amp=0.5, width2=0.05, cx=0.4, cy=0.6), 0.0, 0.05),
])
def test_subdomain_rect_against_oracle(fk, px, py, N, dens, t_w, D):
    """px x py splits (sub-domains wider than tall and taller than wide)."""
    import torch
    xi0, eta0 = prev_mesh(N)
    rng = np.random.default_rng(px * 1000 + py * 10 + N)
    ij = S.interface_index_rect(px, py, N)
    assert len(ij) == fk.n_interface_nodes_rect(px, py, N)
    ix = xi0[ij[:, 1], ij[:, 0]] + 1e-3 * rng.standard_normal(len(ij))
    iy = eta0[ij[:, 1], ij[:, 0]] + 1e-3 * rng.standard_normal(len(ij))
    print(f"[gpu] subdomain rect px={px} py={py} N={N} kind={dens.kind}", flush=True)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    gx, gy = fk.subdomain_solve_rect(dens, t_w, D, px, py, N, cuda(xi0), cuda(eta0), cuda(ix) if len(ij) else e,
                                     cuda(iy) if len(ij) else e)
    torch.cuda.synchronize()
    ox, oy = S.subdomain_be_step_rect(dens, t_w, D, px, py, N, xi0, eta0, ix, iy)
    err = max(np.abs(gx.cpu().numpy() - ox).max(), np.abs(gy.cpu().numpy() - oy).max())
    print(f"max |gpu - oracle| = {err:.3e}", flush=True)
    assert err < 1e-12
    if (px, py) == (8, 6):
        # the exact domain-decomposition identity at full size
        gxi, geta = S.global_be_step(dens, t_w, D, N, xi0, eta0)
        sx, sy = fk.subdomain_solve_rect(dens, t_w, D, px, py, N, cuda(xi0), cuda(eta0),
                                         cuda(gxi[ij[:, 1], ij[:, 0]]), cuda(geta[ij[:, 1], ij[:, 0]]))
        torch.cuda.synchronize()
        assert np.abs(sx.cpu().numpy() - gxi).max() < 1e-12 and np.abs(sy.cpu().numpy() - geta).max() < 1e-12


@pytest.mark.parametrize("px,m,dens,t_w,D", [
    (2, 20, W.paper_ring(W.TIME_FROZEN, 0.3), 0.3, 1e-3),   # the paper's 41 x 41 grid, 2 x 2 layout
    (4, 8, W.ridge(), 0.0, 0.01),
    (2, 32, W.two_bumps(W.TIME_FROZEN, 0.02), 0.02, 5e-4),
])
def test_equidistributed_edges_against_oracle(fk, px, m, dens, t_w, D):
    """Outer boundary data from the 1-D equidistribution of w along the
    edges (Sect. 3): GPU Simpson quadrature against adaptive quadrature."""
    import torch
    N = px * m
    xi0, eta0 = prev_mesh(N)
    ij = S.interface_index(px, m)
    ix, iy = xi0[ij[:, 1], ij[:, 0]], eta0[ij[:, 1], ij[:, 0]]
    print(f"[gpu] subdomain equidistributed edges px={px} m={m} kind={dens.kind}", flush=True)
    gx, gy = fk.subdomain_solve(dens, t_w, D, px, m, cuda(xi0), cuda(eta0), cuda(ix), cuda(iy),
                                bdry_kind=W.DATA_EQUIDISTRIBUTED)
    torch.cuda.synchronize()
    ox, oy = S.subdomain_be_step(dens, t_w, D, px, m, xi0, eta0, ix, iy, bdry="equidistributed")
    err = max(np.abs(gx.cpu().numpy() - ox).max(), np.abs(gy.cpu().numpy() - oy).max())
    print(f"max |gpu - oracle| = {err:.3e}", flush=True)
    assert err < 1e-11


def test_domain_decomposition_identity_on_gpu(fk):
    import torch
    px, m = 4, 16
    N = px * m
    dens = W.moving_bump()
    xi0, eta0 = prev_mesh(N)
    gxi, geta = S.global_be_step(dens, 0.02, 0.01, N, xi0, eta0)
    ij = S.interface_index(px, m)
    sx, sy = fk.subdomain_solve(dens, 0.02, 0.01, px, m, cuda(xi0), cuda(eta0), cuda(gxi[ij[:, 1], ij[:, 0]]),
                                cuda(geta[ij[:, 1], ij[:, 0]]))
    torch.cuda.synchronize()
    assert np.abs(sx.cpu().numpy() - gxi).max() < 1e-12 and np.abs(sy.cpu().numpy() - geta).max() < 1e-12


def test_zero_boundary_sine_mode(fk):
    import torch
    px, m, D = 2, 12, 0.01
    N = px * m
    X, Y = grid(N)
    phi = np.sin(math.pi * X) * np.sin(math.pi * Y)
    h = 1.0 / N
    factor = 1.0 / (1.0 + D * 8.0 / h ** 2 * math.sin(math.pi * h / 2) ** 2)
    ij = S.interface_index(px, m)
    iv = factor * phi[ij[:, 1], ij[:, 0]]
    sx, sy = fk.subdomain_solve(W.CONST, 0.0, D, px, m, cuda(phi), cuda(phi), cuda(iv), cuda(iv),
                                bdry_kind=W.DATA_ZERO)
    torch.cuda.synchronize()
    assert np.abs(sx.cpu().numpy() - factor * phi).max() < 1e-13


@pytest.mark.parametrize("n", [16, 257, 768])
def test_mesh_quality_against_oracle(fk, n):
    import torch
    xi, eta = prev_mesh(n)
    q = fk.fk_mesh_quality(cuda(xi), cuda(eta))
    torch.cuda.synchronize()
    ref = S.mesh_quality(xi, eta)
    assert np.allclose(q.cpu().numpy(), ref, rtol=0, atol=1e-12)
    X, Y = grid(n)
    q = fk.fk_mesh_quality(cuda(X), cuda(Y)).cpu().numpy()
    assert abs(q[0] - 1) < 1e-12 and q[1] < 1e-12
    # a folded map (eta reversed): every Jacobian is -1, and a second call
    # into the same output starts afresh
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    fk.fk_mesh_quality(cuda(X), cuda(Y), out=out)
    fk.fk_mesh_quality(cuda(X), cuda(1.0 - Y), out=out)
    q = out.cpu().numpy()
    ref = S.mesh_quality(X, 1.0 - Y)
    assert abs(q[0] + 1) < 1e-12 and abs(q[0] - ref[0]) < 1e-12 and q[1] < 1e-12
