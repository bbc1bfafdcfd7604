"""TEST INFRASTRUCTURE -- FP64 oracle of key-point placement on the interfaces
and of the piecewise cubic Hermite interpolation of the other interface nodes
(Sect. 4, further speed-up; Sect. 5 uses both in the paper's run).

The paper computes the stochastic solution only near the maxima and minima
of rho_x and rho_xx along the horizontal interfaces (rho_y, rho_yy along the
vertical ones) and recovers the remaining interface points by piecewise
cubic Hermite interpolation.  Readings taken here (the paper says no more):

* rho = 1/w, sampled at the grid nodes of each interface line at the step's
  density time; its derivatives along the line by central differences at
  the line's interior nodes (k = 1 .. N-1), taken unscaled:
  f1_k = rho_{k+1} - rho_{k-1},  f2_k = (rho_{k+1} + rho_{k-1}) - 2 rho_k;
* a key point is a node k (2 <= k <= N-2) where f1 or f2 has a discrete
  extremum -- f_k > f_{k-1} and f_k >= f_{k+1}, or f_k < f_{k-1} and
  f_k <= f_{k+1} -- of size |f_k| >= tol max_k |f_k| (tol screens out the
  round-off ripples of flat stretches);
* the nodes where interface lines cross are always key points (both lines
  interpolate through them);
* no two consecutive knots (key points and the line's two boundary ends)
  are more than max_gap nodes apart: a longer gap of g nodes gets
  q - 1 = ceil(g / max_gap) - 1 further key points at a + floor(r g / q);
* the interpolant on each line passes through the boundary data at its two
  ends and the Monte-Carlo values at its key points, parametrised by the
  node coordinate; it is the monotone piecewise cubic Hermite interpolant of
  Fritsch & Carlson (SIAM J. Numer. Anal. 17, 1980) with the slopes of
  Fritsch & Butland (SIAM J. Sci. Stat. Comput. 5, 1984): at an interior
  knot 0 where the neighbouring secants differ in sign, else their weighted
  harmonic mean with weights (2 h_k + h_{k-1}, h_k + 2 h_{k-1}); at the
  ends the three-point formula ((2 h_0 + h_1) d_0 - h_0 d_1) / (h_0 + h_1),
  set to 0 if its sign differs from d_0's and limited to 3 d_0 where the
  secants change sign; two knots give the straight line.

Only tests use this module.
"""
from __future__ import annotations

import numpy as np

import oracle.subdomain as _sub


def _lines(px, m):
    """Per interface line: (orientation, fixed grid index); vertical lines first."""
    return [("v", a * m) for a in range(1, px)] + [("h", c * m) for c in range(1, px)]


def _index_map(px, m):
    ij = _sub.interface_index(px, m)
    return {(int(i), int(j)): k for k, (i, j) in enumerate(ij)}


def _node(orient, fixed, k):
    """Grid node (i, j) of position k on a line."""
    return (fixed, k) if orient == "v" else (k, fixed)


def line_keys(rho, m, tol, max_gap):
    """Key positions (sorted, 1 .. N-1) on one line from rho at its nodes 0 .. N."""
    rho = np.asarray(rho, dtype=np.float64)
    N = rho.size - 1
    keys = {k for k in range(1, N) if k % m == 0}
    f1 = rho[2:] - rho[:-2]                                  # f[k - 1] belongs to node k
    f2 = (rho[2:] + rho[:-2]) - (rho[1:-1] + rho[1:-1])
    for f in (f1, f2):
        thr = tol * np.abs(f).max()
        if not thr > 0.0:
            continue
        for k in range(2, N - 1):
            fl, fk, fr = f[k - 2], f[k - 1], f[k]
            if abs(fk) >= thr and ((fk > fl and fk >= fr) or (fk < fl and fk <= fr)):
                keys.add(k)
    knots = sorted(keys | {0, N})
    for a, b in zip(knots[:-1], knots[1:]):
        g = b - a
        if g > max_gap:
            q = -(-g // max_gap)
            keys.update(a + (r * g) // q for r in range(1, q))
    return sorted(keys)


def key_mask(w_grid, px, m, tol=1e-2, max_gap=None):
    """Boolean mask over the canonical interface nodes: True at key points.
    w_grid: [(N+1), (N+1)] samples of w indexed [j, i]."""
    w_grid = np.asarray(w_grid, dtype=np.float64)
    max_gap = max_gap or max(1, m // 2)
    idx = _index_map(px, m)
    N = px * m
    mask = np.zeros(len(idx), dtype=bool)
    for orient, fixed in _lines(px, m):
        w_line = w_grid[:, fixed] if orient == "v" else w_grid[fixed, :]
        for k in line_keys(1.0 / w_line, m, tol, max_gap):
            mask[idx[_node(orient, fixed, k)]] = True
    return mask


def pchip_slopes(x, y):
    """Knot slopes of the monotone piecewise cubic Hermite interpolant."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    h = np.diff(x)
    d = np.diff(y) / h
    n = x.size
    s = np.zeros(n)
    if n == 2:
        s[:] = d[0]
        return s
    for k in range(1, n - 1):
        if d[k - 1] * d[k] > 0.0:
            w1, w2 = 2.0 * h[k] + h[k - 1], h[k] + 2.0 * h[k - 1]
            s[k] = (w1 + w2) / (w1 / d[k - 1] + w2 / d[k])

    def end(h0, h1, d0, d1):
        v = ((2.0 * h0 + h1) * d0 - h0 * d1) / (h0 + h1)
        if np.sign(v) != np.sign(d0):
            return 0.0
        if np.sign(d0) != np.sign(d1) and abs(v) > abs(3.0 * d0):
            return 3.0 * d0
        return v

    s[0] = end(h[0], h[1], d[0], d[1])
    s[-1] = end(h[-1], h[-2], d[-1], d[-2])
    return s


def pchip(x, y, xq):
    """The interpolant through (x, y) (x increasing) at the points xq."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xq = np.asarray(xq, dtype=np.float64)
    s = pchip_slopes(x, y)
    k = np.clip(np.searchsorted(x, xq, side="right") - 1, 0, x.size - 2)
    h = x[k + 1] - x[k]
    t = (xq - x[k]) / h
    h00 = (1 + 2 * t) * (1 - t) ** 2
    h10 = t * (1 - t) ** 2
    h01 = t * t * (3 - 2 * t)
    h11 = t * t * (t - 1)
    return h00 * y[k] + h10 * h * s[k] + h01 * y[k + 1] + h11 * h * s[k + 1]


def interpolate_interface(px, m, mask, key_values, edge_xi, edge_eta):
    """Interface values in canonical order: the key points' values
    (key_values [n_keys, 2], in canonical order of the keys), the others by
    the interpolant along their line through the line's boundary ends (from
    the grids edge_xi / edge_eta, whose edge nodes hold the boundary data)
    and its key points."""
    idx = _index_map(px, m)
    N = px * m
    mask = np.asarray(mask, dtype=bool)
    key_values = np.asarray(key_values, dtype=np.float64).reshape(-1, 2)
    slot = np.full(mask.size, -1, dtype=np.int64)
    slot[mask] = np.arange(int(mask.sum()))
    out = np.full((mask.size, 2), np.nan)
    out[mask] = key_values
    grids = (np.asarray(edge_xi, dtype=np.float64), np.asarray(edge_eta, dtype=np.float64))
    for orient, fixed in _lines(px, m):
        kx, others = [], []
        vals = [[], []]
        for k in range(N + 1):
            i, j = _node(orient, fixed, k)
            if k in (0, N):
                kx.append(k / N)
                for c in range(2):
                    vals[c].append(grids[c][j, i])
                continue
            g = idx[(i, j)]
            if slot[g] >= 0:
                kx.append(k / N)
                for c in range(2):
                    vals[c].append(key_values[slot[g], c])
            elif not (orient == "h" and k % m == 0):
                others.append((k, g))
        if not others:
            continue
        q = np.array([k for k, _ in others], dtype=np.float64) / N
        rows = [g for _, g in others]
        for c in range(2):
            out[rows, c] = pchip(kx, vals[c], q)
    if np.isnan(out).any():
        raise AssertionError("an interface node was neither a key point nor interpolated")
    return out


def key_points(w_grid, px, m, tol=1e-2, max_gap=None):
    """(mask, key coordinates [n_keys, 2]) for px x px sub-domains."""
    mask = key_mask(w_grid, px, m, tol, max_gap)
    pts = _sub.interface_index(px, m)[mask].astype(np.float64) / (px * m)
    return mask, pts
