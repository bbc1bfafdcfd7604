"""Pins of the Monte-Carlo oracle against facts the mathematics fixes.

Each test is chosen so that a plausible slip in the oracle -- a dropped
term, a wrong sign, a missing sqrt(2), a wrong step count, a misplaced exit
test or time argument -- fails at least one of them:

* one step (K = 1) with identity data: E[X_1] = P + b(P) D and
  Var[X_1] = 2 D per component, with b = -grad ln w taken by central finite
  differences of the density (drift sign, drift scale, the sqrt(2) factor);
* w = 1, identity data: the stopped chain is a martingale and unclamped
  scoring makes E = P exact for any dt; z-scores over 32 seeds are N(0,1);
* w = 1, sine mode: exp(2 pi^2 s_k) phi(X_k) is an exact discrete martingale,
  so E = exp(-2 pi^2 t) phi(P) for any dt (exit test, scoring, the time of
  the boundary data, the short last step);
* w = w(x): eta = y exactly; a ridge symmetric about x = 1/2 gives xi(1/2, y) = 1/2;
* the static-bump workload against the independent finite-difference solution
  of the PDE (tests/golden), within 4 standard errors plus the time-step bias;
* invariants: estimates in [0, 1], eta non-decreasing up the vertical interface.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

import workloads as W

THREADS = min(8, os.cpu_count() or 1)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def grad_log_w(oracle_mod, dens, tau, pts, h=1e-6):
    """-grad ln w by central differences of the oracle's density w."""
    b = np.zeros_like(pts)
    for c in range(2):
        e = np.zeros(2)
        e[c] = h
        wp, _ = oracle_mod.density(dens, tau, pts + e)
        wm, _ = oracle_mod.density(dens, tau, pts - e)
        b[:, c] = -(np.log(wp) - np.log(wm)) / (2 * h)
    return b


@pytest.mark.parametrize("dens", [W.static_bump(), W.moving_bump(), W.two_bumps(W.TIME_BACKWARD), W.ridge(),
                                  W.paper_ring(W.TIME_BACKWARD)],
                         ids=["bump", "moving", "two", "ridge", "ring"])
def test_drift_is_minus_grad_log_w(oracle_mod, dens):
    pts = W.uniform_points(50, seed=3)
    for tau in (0.0, 0.037, 0.3):
        _, b = oracle_mod.density(dens, tau, pts)
        assert np.allclose(b, grad_log_w(oracle_mod, dens, tau, pts), rtol=1e-6, atol=1e-6)


def test_ring_special_values(oracle_mod):
    # the paper's ring (Sect. 5): w = 1/rho, rho = 1 + 10 exp(-50 |r^2 - 1/100|);
    # on the ring r = 1/10 rho = 11, at the moving centre rho = 1 + 10 exp(-1/2)
    ring = W.paper_ring(W.TIME_BACKWARD)
    tau = 0.2
    c = (0.5 + 0.25 * math.cos(2 * math.pi * tau), 0.5 + 0.25 * math.sin(2 * math.pi * tau))
    w, b = oracle_mod.density(ring, tau, [[c[0], c[1]], [c[0] + 0.1, c[1]], [c[0], c[1] - 0.1]])
    assert w[0] == pytest.approx(1 / (1 + 10 * math.exp(-0.5)), rel=1e-14) and np.allclose(b[0], 0.0)
    assert w[1] == pytest.approx(1 / 11, rel=1e-12) and w[2] == pytest.approx(1 / 11, rel=1e-12)


def test_density_special_values(oracle_mod):
    # static bump peaks at its centre with w = 1 + A
    w, b = oracle_mod.density(W.static_bump(), 0.0, [[0.3, 0.6]])
    assert w[0] == pytest.approx(11.0) and np.allclose(b, 0.0)
    # one width away: 1 + A / e
    w, _ = oracle_mod.density(W.static_bump(), 0.0, [[0.3 + 0.1, 0.6]])
    assert w[0] == pytest.approx(1 + 10 / math.e)
    # moving bump: centre at (3/4, 1/2) at tau = 0 and (1/2, 3/4) at tau = 1/4
    w, _ = oracle_mod.density(W.moving_bump(), 0.0, [[0.75, 0.5]])
    assert w[0] == pytest.approx(21.0)
    w, _ = oracle_mod.density(W.moving_bump(), 0.25, [[0.5, 0.75]])
    assert w[0] == pytest.approx(21.0)
    # two bumps: mirror images in x = 1/2 at every time
    p = np.array([[0.7, 0.55]])
    for tau in (0.0, 0.1, 0.21):
        w1, b1 = oracle_mod.density(W.two_bumps(W.TIME_BACKWARD), tau, p)
        w2, b2 = oracle_mod.density(W.two_bumps(W.TIME_BACKWARD), tau, [[1 - p[0, 0], p[0, 1]]])
        assert w1[0] == pytest.approx(w2[0]) and b1[0, 0] == pytest.approx(-b2[0, 0]) and b1[0, 1] == pytest.approx(b2[0, 1])
    # ridge: no y-drift
    _, b = oracle_mod.density(W.ridge(), 0.0, W.uniform_points(20, seed=1))
    assert np.all(b[:, 1] == 0.0)


def test_step_count(oracle_mod):
    assert oracle_mod.n_steps(0.05, 1e-4) == 500
    assert oracle_mod.n_steps(0.1, 1e-5) == 10000
    assert oracle_mod.n_steps(1.05e-3, 1e-4) == 11
    assert oracle_mod.n_steps(0.0, 1e-4) == 0


@pytest.mark.parametrize("dens,pts", [
    (W.static_bump(), [[0.5, 0.5], [0.42, 0.66], [0.2, 0.55], [0.33, 0.57]]),
    (W.moving_bump(), [[0.7, 0.5], [0.78, 0.45], [0.72, 0.56], [0.8, 0.52]]),
], ids=["bump", "moving"])
def test_one_step_mean_and_variance(oracle_mod, dens, pts):
    """K = 1: X_1 = P + b(t, P) D + sqrt(2 D) z, scored unclamped either way."""
    pts = np.array(pts)
    D = 2e-3
    n = 200_000
    o = oracle_mod.fk_solve(dens, W.Data(), pts, D, D, n, seed=9, threads=THREADS)
    b = grad_log_w(oracle_mod, dens, D, pts)       # BACKWARD: w at PDE time t - 0 = D
    expect = pts + b * D
    assert np.all(np.abs(o["mean"] - expect) <= 4 * o["se"])
    # per-component variance 2 D  -> se = sqrt(2 D / n)
    assert np.allclose(o["se"], math.sqrt(2 * D / n), rtol=0.01)
    # the drift is resolved: it is many standard errors away from zero
    assert np.max(np.abs(b * D) / o["se"]) > 20


def test_const_identity_martingale_over_seeds(oracle_mod):
    pts = np.array([[0.5, 0.5], [0.1, 0.8], [0.93, 0.07], [0.3, 0.35]])
    z = []
    for seed in range(32):
        o = oracle_mod.fk_solve(W.CONST, W.Data(), pts, 0.06, 3e-3, 1500, seed=seed, threads=THREADS)
        z.append(((o["mean"] - pts) / o["se"]).ravel())
    z = np.concatenate(z)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert np.all(np.abs(z) < 5)


@pytest.mark.parametrize("dt", [1e-2, 1e-3])
def test_const_sin_mode_exact_any_dt(oracle_mod, dt):
    pts = W.uniform_points(12, seed=8)
    t = 0.045   # with dt = 1e-2: four steps and a short last one
    data = W.Data(init_kind=W.DATA_SIN, bdry_kind=W.DATA_SIN)
    o = oracle_mod.fk_solve(W.CONST, data, pts, t, dt, 40_000, seed=4, threads=THREADS)
    exact = math.exp(-2 * math.pi ** 2 * t) * np.sin(math.pi * pts[:, 0]) * np.sin(math.pi * pts[:, 1])
    assert np.all(np.abs(o["mean"][:, 0] - exact) <= 4 * o["se"][:, 0])
    assert np.array_equal(o["mean"][:, 0], o["mean"][:, 1])


def test_ridge_eta_exact_and_symmetry(oracle_mod):
    dens = W.ridge(amp=10.0, width2=0.01, cx=0.5)
    ys = np.array([0.2, 0.45, 0.7])
    pts = np.stack([np.full(3, 0.5), ys], 1)
    o = oracle_mod.fk_solve(dens, W.Data(), pts, 0.05, 1e-4, 20_000, seed=2, threads=THREADS)
    assert np.all(np.abs(o["mean"][:, 1] - ys) <= 4 * o["se"][:, 1])
    assert np.all(np.abs(o["mean"][:, 0] - 0.5) <= 4 * o["se"][:, 0])
    # off-centre ridge: the drift pushes xi away from the ridge measurably
    dens2 = W.ridge(amp=10.0, width2=0.01, cx=0.35)
    o2 = oracle_mod.fk_solve(dens2, W.Data(), [[0.42, 0.5]], 0.05, 1e-4, 20_000, seed=2, threads=THREADS)
    assert o2["mean"][0, 0] - 0.42 > 8 * o2["se"][0, 0]


def test_static_bump_against_fd_reference(oracle_mod):
    fd = np.loadtxt(os.path.join(GOLDEN, "static_bump_31_fd.txt"))
    wl = W.STATIC_BUMP_31
    pts = wl.nodes()
    assert np.allclose(fd[:, :2], pts)
    sel = np.array([13, 15, 17, 18, 20, 22])
    o = oracle_mod.fk_solve(wl.density, wl.data, pts[sel], wl.t, wl.dt, 40_000, seed=1, node_ids=sel,
                            threads=THREADS)
    d = np.abs(o["mean"] - fd[sel, 2:4])
    assert np.all(d <= 4 * o["se"] + 1e-3)
    # the reference itself is resolved far below the comparison tolerance
    assert fd[:, 4:].max() < 1e-5


def test_invariants_static_bump(oracle_mod):
    wl = W.STATIC_BUMP_31
    o = oracle_mod.fk_solve(wl.density, wl.data, wl.nodes(), wl.t, wl.dt, wl.n_paths, threads=THREADS)
    m, s = o["mean"], o["se"]
    assert np.all(m >= -3 * s) and np.all(m <= 1 + 3 * s)
    de = np.diff(m[:, 1])
    assert np.all(de >= -3 * np.sqrt(s[1:, 1] ** 2 + s[:-1, 1] ** 2))


def test_zero_horizon_and_exit_records(oracle_mod):
    pts = np.array([[0.25, 0.5], [1.0, 0.5]])
    o = oracle_mod.fk_solve(W.static_bump(), W.Data(), pts, 0.0, 1e-4, 8, want_exit=True, want_scores=True)
    assert np.array_equal(o["mean"], pts) and np.all(o["se"] == 0) and np.all(o["exit_step"] == -1)
    o = oracle_mod.fk_solve(W.static_bump(), W.Data(), pts, 1e-3, 1e-4, 64, want_exit=True, want_scores=True)
    ex, sc = o["exit_step"], o["scores"]
    assert np.all((ex == -1) | ((ex >= 1) & (ex <= 10)))
    out = ex > 0
    # exited paths score a point outside the closed square, survivors one inside
    outside = (sc[..., 0] < 0) | (sc[..., 0] > 1) | (sc[..., 1] < 0) | (sc[..., 1] > 1)
    assert np.array_equal(outside, out)
    # a node on the boundary exits within a few steps on most paths
    assert out[1].mean() > 0.6
    # individual paths agree with the full solve
    sc1, ex1 = oracle_mod.fk_paths(W.static_bump(), W.Data(), pts[[1, 1, 0]], [1, 1, 0], [3, 63, 17], 1e-3, 1e-4)
    assert np.array_equal(ex1, [ex[1, 3], ex[1, 63], ex[0, 17]])
    assert np.array_equal(sc1, sc[[1, 1, 0], [3, 63, 17]])
