"""TEST INFRASTRUCTURE -- FP64 SciPy oracle of the deterministic sub-domain
solves and of the mesh-quality measures.

Deterministic single-domain solver (Sect. 4): the interface values found by
the stochastic solver are Dirichlet data for an implicit finite-difference
discretisation of the relaxed Winslow system (Sect. 2, eq. (3)), solved by
LU factorisation.  Reading taken here (the paper gives no more detail): one
backward-Euler step per mesh step,

    (u^{n+1} - u^n) / D = L_h u^{n+1},
    L_h u = (u_E + u_W + u_N + u_S - 4 u_P) / h^2
            + b_x (u_E - u_W) / (2h) + b_y (u_N - u_S) / (2h),

with b = -grad w / w (eq. (6)) at the node, w held at one time t_w over the
step (Sect. 4 freezes the density over a mesh step), on the uniform nodal
grid x = i/N, y = j/N.  Outer boundary data: the identity (xi = x, eta = y),
zero, or the paper's equidistributed edges (Sect. 3).  ``global_be_step`` solves the whole grid; ``subdomain_be_step``
solves each of px x px sub-domains (m cells a side, N = px m), and
``subdomain_be_step_rect`` each of px x py sub-domains of (N/px) x (N/py)
cells, with the interface nodes as Dirichlet data.  All use scipy.sparse
LU (splu).

Grids are [(N+1), (N+1)] arrays indexed [j, i].
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle as _oracle


def _drift_grid(dens, t_w, N):
    x = np.arange(N + 1) / N
    X, Y = np.meshgrid(x, x)
    pts = np.stack([X.ravel(), Y.ravel()], 1)
    _, b = _oracle.density(dens, t_w, pts)
    return b[:, 0].reshape(N + 1, N + 1), b[:, 1].reshape(N + 1, N + 1)


def _edge_equidistribution(dens, t_w, s, edge, horizontal):
    """int_0^s w / int_0^1 w along the edge y = edge (horizontal) or x = edge."""
    import scipy.integrate as si

    def w(u):
        p = np.array([[u, edge]] if horizontal else [[edge, u]], dtype=np.float64)
        return float(_oracle.density(dens, t_w, p)[0][0])

    kw = dict(epsabs=1e-14, epsrel=1e-13, limit=400)
    if dens.w_grid is None:
        return si.quad(w, 0.0, s, **kw)[0] / si.quad(w, 0.0, 1.0, **kw)[0]
    # a grid density is piecewise linear along the edge: split at its nodes
    n = dens.w_n
    kw["limit"] = max(400, 8 * n)

    def integral(b):
        brk = [k / n for k in range(1, n) if k / n < b]
        return si.quad(w, 0.0, b, points=brk or None, **kw)[0]

    return integral(s) / integral(1.0)


def boundary_grid(N, bdry: str = "identity", dens=None, t_w=0.0):
    """Grids holding the outer boundary data (interior entries unspecified = 0).

    "equidistributed" (Sect. 3): xi = 0 / 1 on the left / right edges, eta = 0
    / 1 on the bottom / top edges, and on the other edges the 1-D version of
    eq. (2), whose solution is xi(x) = int_0^x w / int_0^1 w, for w frozen at
    t_w (adaptive quadrature)."""
    x = np.arange(N + 1) / N
    X, Y = np.meshgrid(x, x)
    gx, gy = np.zeros_like(X), np.zeros_like(X)
    if bdry == "identity":
        for g, v in ((gx, X), (gy, Y)):
            g[0, :], g[-1, :], g[:, 0], g[:, -1] = v[0, :], v[-1, :], v[:, 0], v[:, -1]
    elif bdry == "equidistributed":
        gx[:, -1] = 1.0
        gy[-1, :] = 1.0
        for i in range(1, N):
            gx[0, i] = _edge_equidistribution(dens, t_w, x[i], 0.0, True)
            gx[-1, i] = _edge_equidistribution(dens, t_w, x[i], 1.0, True)
        for j in range(1, N):
            gy[j, 0] = _edge_equidistribution(dens, t_w, x[j], 0.0, False)
            gy[j, -1] = _edge_equidistribution(dens, t_w, x[j], 1.0, False)
    return gx, gy


def _be_solve_region(bx, by, D, h, i0, i1, j0, j1, rhs_grids, bc_grids):
    """Backward-Euler solve on the interior nodes i0 < i < i1, j0 < j < j1;
    every node on the region's edge is Dirichlet data from bc_grids.  With
    D = inf the steady problem -L_h u = 0 (the elliptic system, eq. (2)):
    rows (4 u_P - sum of neighbours) / h^2 - b . grad_h u = 0, no previous
    values."""
    ni, nj = i1 - i0 - 1, j1 - j0 - 1
    n = ni * nj
    idx = lambda i, j: (j - j0 - 1) * ni + (i - i0 - 1)  # noqa: E731
    rows, cols, vals = [], [], []
    rhs = [np.zeros(n) for _ in rhs_grids]
    steady = bool(np.isinf(D))
    scale = 1.0 if steady else D          # the steady rows are the transient ones divided by D, D -> inf
    c0 = scale / h ** 2
    for j in range(j0 + 1, j1):
        for i in range(i0 + 1, i1):
            r = idx(i, j)
            rows.append(r), cols.append(r), vals.append((0.0 if steady else 1.0) + 4.0 * c0)
            if not steady:
                for k, g in enumerate(rhs_grids):
                    rhs[k][r] += g[j, i]
            cx = scale * bx[j, i] / (2 * h)
            cy = scale * by[j, i] / (2 * h)
            for (ii, jj, coef) in ((i + 1, j, -c0 - cx), (i - 1, j, -c0 + cx),
                                   (i, j + 1, -c0 - cy), (i, j - 1, -c0 + cy)):
                if i0 < ii < i1 and j0 < jj < j1:
                    rows.append(r), cols.append(idx(ii, jj)), vals.append(coef)
                else:
                    for k, g in enumerate(bc_grids):
                        rhs[k][r] -= coef * g[jj, ii]
    A = sp.csc_matrix((vals, (rows, cols)), shape=(n, n))
    lu = spla.splu(A)
    return [lu.solve(v).reshape(nj, ni) for v in rhs]


def global_be_step(dens, t_w, D, N, xi_n, eta_n, bdry="identity"):
    """One backward-Euler step on the whole grid (D = inf: the steady solve;
    xi_n, eta_n are then not read)."""
    h = 1.0 / N
    bx, by = _drift_grid(dens, t_w, N)
    gx, gy = boundary_grid(N, bdry, dens, t_w)
    sx, sy = _be_solve_region(bx, by, D, h, 0, N, 0, N, [xi_n, eta_n], [gx, gy])
    xi, eta = gx.copy(), gy.copy()
    xi[1:N, 1:N], eta[1:N, 1:N] = sx, sy
    return xi, eta


def interface_index_rect(px, py, N):
    """Grid indices (i, j) of the interface nodes of a px x py split of the
    N-cell grid in canonical order: vertical lines x = a/px (y ascending),
    then horizontal lines y = c/py (x ascending) without the crossings."""
    mx, my = N // px, N // py
    out = []
    for a in range(1, px):
        for j in range(1, N):
            out.append((a * mx, j))
    for c in range(1, py):
        for i in range(1, N):
            if i % mx == 0:
                continue
            out.append((i, c * my))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


def interface_index(px, m):
    """The same for px x px sub-domains of m cells a side (N = px m)."""
    return interface_index_rect(px, px, px * m)


def subdomain_be_step_rect(dens, t_w, D, px, py, N, xi_n, eta_n, iface_xi, iface_eta, bdry="identity"):
    """Backward-Euler step on each of px x py sub-domains of (N/px) x (N/py)
    cells with the interface values (canonical order) as Dirichlet data;
    returns the assembled grids."""
    assert N % px == 0 and N % py == 0
    mx, my = N // px, N // py
    h = 1.0 / N
    bx, by = _drift_grid(dens, t_w, N)
    xi, eta = boundary_grid(N, bdry, dens, t_w)
    ij = interface_index_rect(px, py, N)
    if len(ij):
        xi[ij[:, 1], ij[:, 0]] = iface_xi
        eta[ij[:, 1], ij[:, 0]] = iface_eta
    for sj in range(py):
        for si in range(px):
            i0, i1, j0, j1 = si * mx, (si + 1) * mx, sj * my, (sj + 1) * my
            sx, sy = _be_solve_region(bx, by, D, h, i0, i1, j0, j1, [xi_n, eta_n], [xi, eta])
            xi[j0 + 1:j1, i0 + 1:i1], eta[j0 + 1:j1, i0 + 1:i1] = sx, sy
    return xi, eta


def subdomain_be_step(dens, t_w, D, px, m, xi_n, eta_n, iface_xi, iface_eta, bdry="identity"):
    """Backward-Euler step on each of px x px sub-domains (m cells a side)."""
    return subdomain_be_step_rect(dens, t_w, D, px, px, px * m, xi_n, eta_n, iface_xi, iface_eta, bdry)


def mesh_quality(xi, eta):
    """(min Jacobian, max skewness) over the cells of a mesh map (xi, eta).

    Cell-centred differences: for the cell with lower-left node (i, j),
    u_x = average of the two x-differences along its bottom and top edges
    over h, u_y likewise; J = xi_x eta_y - xi_y eta_x;
    skew = |grad xi . grad eta| / (|grad xi| |grad eta|).
    """
    N = xi.shape[0] - 1
    h = 1.0 / N

    def grads(u):
        ux = ((u[:-1, 1:] - u[:-1, :-1]) + (u[1:, 1:] - u[1:, :-1])) / (2 * h)
        uy = ((u[1:, :-1] - u[:-1, :-1]) + (u[1:, 1:] - u[:-1, 1:])) / (2 * h)
        return ux, uy

    xx, xy = grads(xi)
    ex, ey = grads(eta)
    J = xx * ey - xy * ex
    skew = np.abs(xx * ex + xy * ey) / (np.hypot(xx, xy) * np.hypot(ex, ey))
    return float(J.min()), float(skew.max())
