"""Pins of the control-variate network oracle: forward-mode derivatives and
backpropagated gradients against finite differences, Adam's first step in
closed form, BF16 rounding, and the C and NumPy evaluations against each
other."""
import numpy as np
import pytest

import oracle.mlp as M
import workloads as W

T = W.CV_T_SCALE


@pytest.fixture(scope="module")
def flat():
    rng = np.random.default_rng(3)
    # larger than the initial scale so that the tanh curvature matters
    return M.bf16_round(W.mlp_init(1) * 2.5 + 0.05 * rng.standard_normal(M.N_PARAMS))


def pts(n=32, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, T, n), rng.uniform(0.05, 0.95, n), rng.uniform(0.05, 0.95, n)


def test_forward_mode_value_matches_forward(flat):
    t, x, y = pts()
    fm = M.forward_mode(flat, t, x, y, T)
    assert np.allclose(fm["val"], M.forward(flat, t, x, y, T), rtol=0, atol=1e-14)


def test_first_derivatives_by_central_differences(flat):
    t, x, y = pts()
    fm = M.forward_mode(flat, t, x, y, T)
    for key, (dt_, dx_, dy_), h in (("dx", (0, 1, 0), 1e-6), ("dy", (0, 0, 1), 1e-6), ("dt", (1, 0, 0), 1e-8)):
        fp = M.forward(flat, t + h * dt_, x + h * dx_, y + h * dy_, T)
        fmn = M.forward(flat, t - h * dt_, x - h * dx_, y - h * dy_, T)
        fd = (fp - fmn) / (2 * h)
        assert np.allclose(fm[key], fd, rtol=1e-6, atol=1e-7), key


def test_laplacian_by_second_differences(flat):
    t, x, y = pts()
    fm = M.forward_mode(flat, t, x, y, T)
    h = 1e-3
    f0 = M.forward(flat, t, x, y, T)
    lap = (M.forward(flat, t, x + h, y, T) + M.forward(flat, t, x - h, y, T) + M.forward(flat, t, x, y + h, T)
           + M.forward(flat, t, x, y - h, T) - 4 * f0) / h ** 2
    scale = np.abs(fm["lap"]).max()
    assert scale > 0.1
    assert np.abs(fm["lap"] - lap).max() < 1e-4 * scale


def test_c_forward_mode_matches_numpy(flat, oracle_mod):
    t, x, y = pts(50, 5)
    c = oracle_mod.mlp_eval_c(flat, T, np.stack([t, x, y], 1))
    fm = M.forward_mode(flat, t, x, y, T)
    for k, key in enumerate(("val", "dx", "dy", "dt", "lap")):
        assert np.allclose(c[:, :, k], fm[key], rtol=1e-12, atol=1e-12), key


def test_backprop_gradient_by_finite_differences(flat):
    rng = np.random.default_rng(11)
    t, x, y = pts(40, 7)
    txy = np.stack([t, x, y], 1)
    target = rng.uniform(0, 1, (40, 2))
    loss, g = M.loss_and_grad(flat, txy, target, T)
    # check a spread of coordinates in every parameter block
    idx = np.concatenate([rng.choice(M.N_PARAMS, 60, replace=False), [0, 200, 256, 4400, 8600, 8705]])
    h = 1e-6
    for i in idx:
        e = np.zeros(M.N_PARAMS)
        e[i] = h
        lp, _ = M.loss_and_grad(flat + e, txy, target, T)
        lm, _ = M.loss_and_grad(flat - e, txy, target, T)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, i
    # and the loss is what it says
    assert loss == pytest.approx(np.mean((M.forward(flat, t, x, y, T) - target) ** 2), rel=1e-14)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(2)
    p = rng.standard_normal(100)
    g = rng.standard_normal(100)
    p1, m, v = M.adam_step(p, g, np.zeros(100), np.zeros(100), 1, 1e-3)
    # bias correction makes m_hat = g, v_hat = g^2: a step of lr * g / (|g| + eps)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, -2.5, 1 + 2 ** -7 + 2 ** -8, 3.0e-3])
    r = M.bf16_round(vals)
    assert r[0] == 1.0 and r[1] == 1.0          # a tie rounds to even
    assert r[2] == 1 + 2 ** -7                   # above the tie rounds up
    assert r[3] == -2.5
    assert r[4] == 1 + 2 ** -6                   # tie at odd rounds up to even
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8
    f = np.asarray(r, dtype=np.float32).view(np.uint32)
    assert np.all(f & 0xFFFF == 0)


def test_init_is_glorot_uniform():
    f = W.mlp_init(0)
    p = M.unflatten(f)
    for name, fan in (("W1", 3 + 64), ("W2", 128), ("W3", 128), ("W4", 66)):
        a = np.sqrt(6.0 / fan)
        assert np.abs(p[name]).max() <= a and np.abs(p[name]).max() > 0.9 * a
    for b in ("b1", "b2", "b3", "b4"):
        assert np.all(p[b] == 0)
    assert np.array_equal(f, W.mlp_init(0))
