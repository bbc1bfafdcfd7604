"""Pins of the control-variate oracle, Dynkin form then martingale form.

* u_hat = 0 reproduces the plain estimate bit for bit.
* w = 1 with the exact solution as u_hat (identity data and u_hat = (x, y);
  the sine mode and u_hat its exact decaying solution): every path scores
  the same number, so the estimate is exact with zero variance, for any dt
  and any stride.
* A linear u_hat with w != 1: the CV estimate agrees with the plain one
  within their standard errors (its integrand b . grad u_hat varies along
  the path, so this is a statistical check only), and the CV variance is
  lower where the drift is strong.
* The quadrature of the Dynkin integral: with w = 1 and the test function
  u_hat = (tau x^2, tau y^2) the integrand's mean is linear in the path
  time, so the trapezoidal rule is exact in expectation and the left-point
  rule is off by 2 sum L_j^2 (L_j the interval lengths); cv - plain on the
  same paths tells the two apart by many standard errors.
* A trained-looking network: CV and plain agree within 3 combined standard
  errors on the same paths.

Martingale form:

* u_hat = 0 reproduces the plain estimate bit for bit.
* w = 1, identity data, grad u_hat = I: every path scores its start point,
  for any stride, with exits and a short last step (the Brownian part is
  accumulated exactly as the path moves).
* w = 1, the sine mode with its exact solution: the remaining variance is
  the stochastic integral's discretisation, falling like sqrt(dt).
* A curved network under a strong drift, strides 2 and 50: cv - plain on the
  same paths has mean zero (z-scores), i.e. no stride bias.
"""
import math

import numpy as np
import pytest

import oracle.mlp as M
import workloads as W


def test_zero_uhat_is_plain(oracle_mod):
    pts = W.uniform_points(6, seed=1)
    cv = oracle_mod.fk_solve_cv(W.static_bump(), W.Data(), pts, 0.02, 1e-4, 500, seed=3, uhat=oracle_mod.UHAT_ZERO)
    pl = oracle_mod.fk_solve(W.static_bump(), W.Data(), pts, 0.02, 1e-4, 500, seed=3)
    assert np.array_equal(cv["mean"], pl["mean"]) and np.array_equal(cv["se"], pl["se"])
    assert np.array_equal(cv["plain_mean"], pl["mean"])


def test_exact_uhat_gives_zero_variance(oracle_mod):
    pts = W.uniform_points(8, seed=2)
    for stride in (1, 3):
        r = oracle_mod.fk_solve_cv(W.CONST, W.Data(), pts, 0.05, 2e-3, 400, seed=1,
                                   uhat=oracle_mod.UHAT_LINEAR, stride=stride)
        assert np.allclose(r["mean"], pts, rtol=0, atol=1e-14) and np.all(r["se"] < 1e-14)
        assert np.all(r["plain_se"] > 1e-3)
        d = W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_SIN)
        r = oracle_mod.fk_solve_cv(W.CONST, d, pts, 0.05, 2e-3, 400, seed=1, uhat=oracle_mod.UHAT_SIN,
                                   stride=stride)
        exact = math.exp(-2 * math.pi ** 2 * 0.05) * np.sin(math.pi * pts[:, 0]) * np.sin(math.pi * pts[:, 1])
        assert np.allclose(r["mean"][:, 0], exact, rtol=0, atol=1e-13) and np.all(r["se"] < 1e-13)


def test_linear_uhat_is_unbiased_with_drift(oracle_mod):
    pts = np.array([[0.35, 0.55], [0.25, 0.62], [0.5, 0.5]])
    r = oracle_mod.fk_solve_cv(W.static_bump(), W.Data(), pts, 0.03, 1e-4, 20000, seed=4,
                               uhat=oracle_mod.UHAT_LINEAR)
    d = np.abs(r["mean"] - r["plain_mean"])
    assert np.all(d <= 3 * np.sqrt(r["se"] ** 2 + r["plain_se"] ** 2))
    # near the bump the CV removes the Brownian part: much lower variance
    assert np.all(r["se"][:2] < 0.5 * r["plain_se"][:2])


@pytest.mark.parametrize("K", [100, 125])
def test_dynkin_trapezoid_exact_for_linear_mean_integrand(oracle_mod, K):
    """w = 1, u_hat = (tau x^2, tau y^2), t_init = 0, nodes far from the
    boundary (a few exits in 10^5 paths).  The integrand r = Laplacian u_hat -
    d_tau u_hat = 2 tau - x^2 has E[r(s)] = 2 (t - s) - (p^2 + 2 s), linear in
    s, so the trapezoidal rule over [0, t] with intervals every `stride` steps
    and the last one closed at the path's end integrates its mean exactly:
    E[estimate - plain] = 0.  The left-point rule would add 2 sum_j L_j^2; a
    missing end interval would drop about L E[r] ~ 6e-4.  Checked per path
    (cv - plain on the same counters) so that the difference's standard error
    (~1.5e-6) resolves the left-point bias (2.5e-5 for K = 100) many times."""
    dt, stride = 5e-5, 50
    t = K * dt
    pts = np.array([[0.5, 0.5], [0.47, 0.53]])
    n = 40000
    cv = oracle_mod.fk_solve_cv(W.CONST, W.Data(), pts, t, dt, n, seed=7, uhat=oracle_mod.UHAT_QUAD,
                                stride=stride, form=oracle_mod.CV_DYNKIN, want_scores=True, want_exit=True)
    pl = oracle_mod.fk_solve(W.CONST, W.Data(), pts, t, dt, n, seed=7, want_scores=True)
    assert np.mean(cv["exit_step"] >= 0) < 2e-4          # almost no path reaches the boundary
    d = cv["cv_scores"] - pl["scores"]                  # -u_hat(end) + integral, per path
    uhat_start = t * pts ** 2                           # u_hat(t, P), added to the CV estimate
    err = d.mean(axis=1) + uhat_start                   # E = 0 for the trapezoidal rule
    se = d.std(axis=1, ddof=1) / np.sqrt(n)
    assert np.all(se < 2.5e-6)
    assert np.all(np.abs(err) <= 4 * se), (err, se)
    # the estimate itself: CV mean minus plain mean on the same paths
    assert np.allclose(cv["mean"] - cv["plain_mean"], err, rtol=0, atol=1e-12)
    lengths = [stride * dt] * (K // stride) + ([(K % stride) * dt] if K % stride else [])
    left_bias = 2.0 * sum(L * L for L in lengths)
    assert left_bias > 10 * se.max()                    # the test separates the two rules
    assert np.all(np.abs(err - left_bias) > 6 * se)


def test_network_uhat_agrees_with_plain(oracle_mod):
    flat = M.bf16_round(W.mlp_init(0))
    pts = np.array([[0.5, 0.3], [0.45, 0.6]])
    r = oracle_mod.fk_solve_cv(W.moving_bump(), W.Data(), pts, 0.01, 1e-4, 400, seed=2,
                               uhat=oracle_mod.UHAT_MLP, flat=flat, t_scale=W.CV_T_SCALE, stride=2)
    d = np.abs(r["mean"] - r["plain_mean"])
    assert np.all(d <= 3 * np.sqrt(r["se"] ** 2 + r["plain_se"] ** 2) + 1e-3)


# ---- martingale form --------------------------------------------------------
# score = g - sum_j grad u_hat(X_{k_j}) . (B_{k_{j+1}} - B_{k_j}), B the
# Brownian part of the Euler-Maruyama path.

def test_martingale_zero_uhat_is_plain(oracle_mod):
    pts = W.uniform_points(6, seed=1)
    cv = oracle_mod.fk_solve_cv(W.static_bump(), W.Data(), pts, 0.02, 1e-4, 500, seed=3,
                                uhat=oracle_mod.UHAT_ZERO, form=oracle_mod.CV_MARTINGALE, stride=4)
    pl = oracle_mod.fk_solve(W.static_bump(), W.Data(), pts, 0.02, 1e-4, 500, seed=3)
    assert np.array_equal(cv["mean"], pl["mean"]) and np.array_equal(cv["se"], pl["se"])


def test_martingale_linear_uhat_w1_is_exact_on_every_path(oracle_mod):
    """w = 1, identity data scored unclamped: g(X_tau) = X_tau = P + B_tau, so
    with grad u_hat = I the score is P on every path, whatever the stride, the
    exits and the short last step (0.05 / 2e-3 is not a whole number of steps
    for 0.051)."""
    pts = W.uniform_points(8, seed=2)
    for stride in (1, 3, 1000):
        r = oracle_mod.fk_solve_cv(W.CONST, W.Data(), pts, 0.051, 2e-3, 400, seed=1, uhat=oracle_mod.UHAT_LINEAR,
                                   stride=stride, form=oracle_mod.CV_MARTINGALE, want_scores=True, want_exit=True)
        assert np.any(r["exit_step"] >= 0)
        assert np.abs(r["cv_scores"] - pts[:, None, :]).max() < 1e-14
        assert np.all(r["plain_se"] > 1e-3)


def test_martingale_exact_sine_solution_removes_the_variance(oracle_mod):
    """With the exact solution's gradient every step, what is left is the
    discretisation of the stochastic integral: the CV standard error falls
    like sqrt(dt) relative to the plain one, and the estimate stays exact."""
    pts = W.uniform_points(6, seed=5)
    d = W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_SIN)
    exact = math.exp(-2 * math.pi ** 2 * 0.05) * np.sin(math.pi * pts[:, 0]) * np.sin(math.pi * pts[:, 1])
    ratio = []
    for dt in (1e-3, 1e-4):
        r = oracle_mod.fk_solve_cv(W.CONST, d, pts, 0.05, dt, 2000, seed=1, uhat=oracle_mod.UHAT_SIN, stride=1,
                                   form=oracle_mod.CV_MARTINGALE)
        assert np.all(np.abs(r["mean"][:, 0] - exact) <= 4 * r["se"][:, 0])
        ratio.append(np.median(r["se"][:, 0] / r["plain_se"][:, 0]))
    assert ratio[1] < 0.08 and 0.25 < ratio[1] / ratio[0] < 0.4     # 1/sqrt(10) = 0.316


def test_martingale_form_is_unbiased_at_any_stride(oracle_mod):
    """The martingale sum has mean zero for the discrete chain, for any
    network and stride: cv - plain on the same paths is a zero-mean sum."""
    flat = M.bf16_round(W.mlp_init(1) * 2.5)
    pts = W.interface_nodes(4, 4, 8)[::2]
    z = []
    for stride in (2, 50):
        r = oracle_mod.fk_solve_cv(W.moving_bump(), W.Data(), pts, 0.01, 1e-4, 1500, seed=6, uhat=oracle_mod.UHAT_MLP,
                                   flat=flat, t_scale=W.CV_T_SCALE, stride=stride, form=oracle_mod.CV_MARTINGALE,
                                   want_scores=True)
        pl = oracle_mod.fk_solve(W.moving_bump(), W.Data(), pts, 0.01, 1e-4, 1500, seed=6, want_scores=True)
        diff = r["cv_scores"] - pl["scores"]
        z.append(diff.mean(1) / (diff.std(1, ddof=1) / math.sqrt(diff.shape[1])))
        assert np.all(np.abs(r["mean"] - diff.mean(1) - pl["mean"]) < 1e-12)
    z = np.concatenate(z).ravel()
    assert np.abs(z).max() < 4.0 and abs(z.mean()) < 4 / math.sqrt(z.size)


# ---- martingale form with the grid initial data as the control ----------------
# G = gradient of the bilinear interpolant of the (xi, eta) grids at the path.

def _nodal(n):
    x = np.arange(n + 1) / n
    return np.meshgrid(x, x)


def test_grid_control_of_the_identity_mesh_is_exact(oracle_mod):
    """The identity mesh's interpolant has gradient I, so under w = 1 with
    identity boundary data every path scores its start point, any stride."""
    X, Y = _nodal(32)
    pts = W.uniform_points(8, seed=9)
    data = W.Data(init_kind=W.DATA_GRID, grid_xi=X, grid_eta=Y)
    for stride in (1, 4, 1000):
        r = oracle_mod.fk_solve_cv(W.CONST, data, pts, 0.051, 2e-3, 300, seed=2, uhat=oracle_mod.UHAT_GRID,
                                   stride=stride, form=oracle_mod.CV_MARTINGALE, want_scores=True, want_exit=True)
        assert np.any(r["exit_step"] >= 0)
        assert np.abs(r["cv_scores"] - pts[:, None, :]).max() < 1e-13


def test_grid_control_is_unbiased_and_reduces_variance(oracle_mod):
    """A deformed mesh under two frozen bumps: cv - plain on the same paths
    has mean zero at strides 2 and 20, and the control removes most of the
    variance."""
    X, Y = _nodal(48)
    xi = X + 0.02 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    eta = Y + 0.015 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    data = W.Data(init_kind=W.DATA_GRID, score_mode=W.SCORE_EXTEND, grid_xi=xi, grid_eta=eta)
    dens = W.two_bumps(W.TIME_FROZEN, 0.01)
    pts = W.interface_nodes(4, 4, 48)[::9]
    pl = oracle_mod.fk_solve(dens, data, pts, 5e-4, 2.5e-5, 2000, seed=4, want_scores=True)
    z = []
    for stride in (2, 20):
        r = oracle_mod.fk_solve_cv(dens, data, pts, 5e-4, 2.5e-5, 2000, seed=4, uhat=oracle_mod.UHAT_GRID,
                                   stride=stride, form=oracle_mod.CV_MARTINGALE, want_scores=True)
        diff = r["cv_scores"] - pl["scores"]
        z.append(diff.mean(1) / (diff.std(1, ddof=1) / math.sqrt(diff.shape[1])))
        ratio = np.median(r["se"] / pl["se"])
        assert ratio < (0.1 if stride == 2 else 0.5), (stride, ratio)
    z = np.concatenate(z).ravel()
    assert np.abs(z).max() < 4.0 and abs(z.mean()) < 4 / math.sqrt(z.size)


def test_grid_control_needs_the_martingale_form(oracle_mod):
    X, Y = _nodal(8)
    data = W.Data(init_kind=W.DATA_GRID, grid_xi=X, grid_eta=Y)
    with pytest.raises(ValueError):
        oracle_mod.fk_solve_cv(W.CONST, data, [[0.5, 0.5]], 0.01, 1e-3, 10, uhat=oracle_mod.UHAT_GRID,
                               form=oracle_mod.CV_DYNKIN)


@pytest.mark.parametrize("form", ["dynkin", "martingale"])
def test_identity_base_is_the_identity_plus_the_network(oracle_mod, form):
    """Both estimator forms are affine in u_hat (the martingale sum and the
    Dynkin terms are linear in it; g enters once), so for any network, per
    path: score(identity + network) = score(network) + score(identity) -
    score(0).  With a zero network the base is the linear control itself."""
    f = oracle_mod.CV_DYNKIN if form == "dynkin" else oracle_mod.CV_MARTINGALE
    dens, pts = W.moving_bump(), W.uniform_points(6, seed=9)
    flat = W.mlp_init(4).astype(np.float64)
    kw = dict(seed=3, stride=4, form=f, want_scores=True, threads=4)

    def run(uhat, fl=None):
        return oracle_mod.fk_solve_cv(dens, W.Data(), pts, 0.01, 1e-3, 300, uhat=uhat, flat=fl, **kw)

    base = run(oracle_mod.UHAT_MLP_BASE, flat)
    net = run(oracle_mod.UHAT_MLP, flat)
    lin = run(oracle_mod.UHAT_LINEAR)
    zero = run(oracle_mod.UHAT_ZERO)
    expect = net["cv_scores"] + lin["cv_scores"] - zero["cv_scores"]
    assert np.abs(base["cv_scores"] - expect).max() < 1e-12
    assert np.abs(base["mean"] - (net["mean"] + lin["mean"] - zero["mean"])).max() < 1e-12
    zero_net = run(oracle_mod.UHAT_MLP_BASE, np.zeros_like(flat))
    assert np.array_equal(zero_net["cv_scores"], lin["cv_scores"])


# ---- martingale form with the network as the deviation from the mesh ---------
# u_hat = bilinear(grid initial data) + MLP: G = grid gradient + network gradient.

def test_grid_base_is_the_grid_plus_the_network(oracle_mod):
    """The martingale score is affine in G, so per path: score(grid + net at
    stride 4) = score(net at stride 4) + score(grid at stride 2) - score(0)
    (the grid part is taken every 2 steps, the network's held over its 4); a
    zero network gives the grid control at stride 2 bitwise; on the identity
    mesh the base is the identity base."""
    X, Y = _nodal(48)
    xi = X + 0.02 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    eta = Y + 0.015 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    data = W.Data(init_kind=W.DATA_GRID, score_mode=W.SCORE_EXTEND, grid_xi=xi, grid_eta=eta)
    dens = W.two_bumps(W.TIME_FROZEN, 0.01)
    pts = W.interface_nodes(4, 4, 48)[::11]
    flat = W.mlp_init(4).astype(np.float64)
    kw = dict(seed=3, stride=4, form=oracle_mod.CV_MARTINGALE, want_scores=True, threads=4)

    def run(uhat, fl=None, d=data, stride=4):
        return oracle_mod.fk_solve_cv(dens, d, pts, 5e-4, 2.5e-5, 300, uhat=uhat, flat=fl, **{**kw, "stride": stride})

    both = run(oracle_mod.UHAT_GRID_MLP, flat)
    expect = run(oracle_mod.UHAT_MLP, flat)["cv_scores"] + run(oracle_mod.UHAT_GRID, stride=2)["cv_scores"] \
        - run(oracle_mod.UHAT_ZERO)["cv_scores"]
    assert np.abs(both["cv_scores"] - expect).max() < 1e-12
    assert np.abs(run(oracle_mod.UHAT_GRID_MLP, np.zeros_like(flat))["cv_scores"]
                  - run(oracle_mod.UHAT_GRID, stride=2)["cv_scores"]).max() < 1e-15
    # on the identity mesh the grid part is I, constant: blocks of 2 or 4 steps
    # give the same sum
    ident = W.Data(init_kind=W.DATA_GRID, score_mode=W.SCORE_EXTEND, grid_xi=X, grid_eta=Y)
    a = run(oracle_mod.UHAT_GRID_MLP, flat, ident)["cv_scores"]
    b = oracle_mod.fk_solve_cv(dens, ident, pts, 5e-4, 2.5e-5, 300, uhat=oracle_mod.UHAT_MLP_BASE, flat=flat,
                               **kw)["cv_scores"]
    assert np.abs(a - b).max() < 1e-12
    with pytest.raises(ValueError):
        oracle_mod.fk_solve_cv(dens, data, pts, 5e-4, 2.5e-5, 10, uhat=oracle_mod.UHAT_GRID_MLP, flat=flat,
                               form=oracle_mod.CV_DYNKIN)


def test_grid_base_control_is_unbiased(oracle_mod):
    """A curved network on top of a deformed mesh: cv - plain on the same
    paths has mean zero (z-scores) at strides 2 and 20."""
    X, Y = _nodal(48)
    xi = X + 0.02 * np.sin(math.pi * X) * np.sin(2 * math.pi * Y)
    eta = Y + 0.015 * np.sin(2 * math.pi * X) * np.sin(math.pi * Y)
    data = W.Data(init_kind=W.DATA_GRID, score_mode=W.SCORE_EXTEND, grid_xi=xi, grid_eta=eta)
    dens = W.two_bumps(W.TIME_FROZEN, 0.01)
    pts = W.interface_nodes(4, 4, 48)[::9]
    flat = M.bf16_round(W.mlp_init(1) * 2.5)
    pl = oracle_mod.fk_solve(dens, data, pts, 5e-4, 2.5e-5, 2000, seed=8, want_scores=True)
    z = []
    for stride in (2, 20):
        r = oracle_mod.fk_solve_cv(dens, data, pts, 5e-4, 2.5e-5, 2000, seed=8, uhat=oracle_mod.UHAT_GRID_MLP,
                                   flat=flat, t_scale=W.CV_T_SCALE, stride=stride, form=oracle_mod.CV_MARTINGALE,
                                   want_scores=True)
        diff = r["cv_scores"] - pl["scores"]
        z.append(diff.mean(1) / (diff.std(1, ddof=1) / math.sqrt(diff.shape[1])))
    z = np.concatenate(z).ravel()
    assert np.abs(z).max() < 4.0 and abs(z.mean()) < 4 / math.sqrt(z.size)


def test_martingale_form_with_the_bridge_test(oracle_mod):
    """The bridge test in the martingale form: the plain part is the plain
    bridge solve on the same counters (identical exits, identical scores);
    with w = 1 and the linear control the CV score differs from the start
    point only by the projection of the last end point onto the square, so
    its mean is the start point (the bridge identity pin), exactly so along
    the near side; with a curved network over a moving density cv - plain
    has mean zero."""
    pts = np.array([[0.03, 0.5], [0.5, 0.04], [0.96, 0.45], [0.55, 0.97], [0.08, 0.3]])
    t = 4e-3
    data = W.Data(score_mode=W.SCORE_BRIDGE)
    pl = oracle_mod.fk_solve(W.CONST, data, pts, t, t / 2, 20000, seed=3, want_exit=True, want_scores=True)
    r = oracle_mod.fk_solve_cv(W.CONST, data, pts, t, t / 2, 20000, seed=3, uhat=oracle_mod.UHAT_LINEAR, stride=2,
                               form=oracle_mod.CV_MARTINGALE, want_scores=True, want_exit=True)
    assert np.array_equal(r["exit_step"], pl["exit_step"])
    assert np.array_equal(r["plain_mean"], pl["mean"]) and np.array_equal(r["plain_se"], pl["se"])
    assert np.all(np.abs(r["mean"] - pts) < 4.5 * r["se"] + 1e-12)   # tangential: x0 to round-off
    assert np.all(r["se"] < pl["se"])
    tangential = np.array([[0, 1], [1, 0], [2, 1], [3, 0]])   # the coordinate along the near side
    assert np.all(r["se"][tangential[:, 0], tangential[:, 1]] < 1e-12)
    # a curved network, a moving density, strides 2 and 10
    dens = W.moving_bump()
    nodes = W.MOVING_BUMP_1521.nodes()[::97]
    flat = M.bf16_round(W.mlp_init(2) * 2.0)
    base = oracle_mod.fk_solve(dens, data, nodes, 0.01, 1e-4, 2000, seed=5, want_scores=True)
    z = []
    for stride in (2, 10):
        c = oracle_mod.fk_solve_cv(dens, data, nodes, 0.01, 1e-4, 2000, seed=5, uhat=oracle_mod.UHAT_MLP, flat=flat,
                                   t_scale=W.CV_T_SCALE, stride=stride, form=oracle_mod.CV_MARTINGALE,
                                   want_scores=True)
        diff = c["cv_scores"] - base["scores"]
        z.append(diff.mean(1) / (diff.std(1, ddof=1) / math.sqrt(diff.shape[1])))
    z = np.concatenate(z).ravel()
    assert np.abs(z).max() < 4.0 and abs(z.mean()) < 4 / math.sqrt(z.size)
    # the Dynkin form does not take the bridge test
    with pytest.raises(Exception):
        oracle_mod.fk_solve_cv(W.CONST, data, pts, t, t / 2, 64, uhat=oracle_mod.UHAT_LINEAR, stride=2,
                               form=oracle_mod.CV_DYNKIN)
