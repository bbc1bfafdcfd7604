"""TEST INFRASTRUCTURE -- FP64 NumPy oracle of the control-variate network.

The network u_hat(t, x, y) -> (xi_hat, eta_hat) is a tanh MLP 3 -> 64 -> 64 ->
64 -> 2 with linear outputs on the normalised input
z = (2 t / T - 1, 2 x - 1, 2 y - 1).  This module evaluates it in FP64 from
a flat parameter vector (the kernels' BF16 values, widened): the plain
forward pass, the forward-mode derivatives the Dynkin-form control variate
needs (value, d/dx, d/dy, d/dt, Laplacian in (x, y)), the mean-squared-error
loss with its gradient by backpropagation, and one Adam step (Kingma & Ba,
2015, with bias correction).  Every derivative is written out by the chain
rule; the tests check them against finite differences.

Flat layout (row-major): W1[64,3] b1[64] W2[64,64] b2[64] W3[64,64] b3[64]
W4[2,64] b4[2]: 8706 numbers.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 64
SHAPES = [("W1", (64, 3)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 64)), ("b3", (64,)),
          ("W4", (2, 64)), ("b4", (2,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(flat):
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def flatten(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16_round(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def normalise(t, x, y, t_scale):
    return np.stack([2.0 * np.asarray(t) / t_scale - 1.0, 2.0 * np.asarray(x) - 1.0, 2.0 * np.asarray(y) - 1.0], 1)


def forward(flat, t, x, y, t_scale):
    """Network outputs [n, 2]."""
    p = unflatten(flat)
    z = normalise(t, x, y, t_scale)
    h = np.tanh(z @ p["W1"].T + p["b1"])
    h = np.tanh(h @ p["W2"].T + p["b2"])
    h = np.tanh(h @ p["W3"].T + p["b3"])
    return h @ p["W4"].T + p["b4"]


def forward_mode(flat, t, x, y, t_scale):
    """Value and derivatives of both outputs: dict of [n, 2] arrays 'val',
    'dx', 'dy', 'dt', 'lap' (lap = d2/dx2 + d2/dy2).

    For a = W h + b and h' = tanh(a): d h' = s d a with s = 1 - h'^2, and
    Laplacian(h') = -2 h' s (|d_x a|^2 + |d_y a|^2) + s Laplacian(a).
    """
    p = unflatten(flat)
    z = normalise(t, x, y, t_scale)
    n = z.shape[0]
    # dz/dt = 2/T, dz/dx = 2, dz/dy = 2 on their own components
    a = z @ p["W1"].T + p["b1"]
    da = {"dt": np.tile(p["W1"][:, 0] * (2.0 / t_scale), (n, 1)),
          "dx": np.tile(p["W1"][:, 1] * 2.0, (n, 1)),
          "dy": np.tile(p["W1"][:, 2] * 2.0, (n, 1))}
    la = np.zeros_like(a)
    for W, b in ((None, None), (p["W2"], p["b2"]), (p["W3"], p["b3"])):
        if W is not None:
            a = h @ W.T + b
            da = {k: v @ W.T for k, v in dh.items()}
            la = lh @ W.T
        h = np.tanh(a)
        s = 1.0 - h * h
        dh = {k: s * v for k, v in da.items()}
        lh = -2.0 * h * s * (da["dx"] ** 2 + da["dy"] ** 2) + s * la
    out = {"val": h @ p["W4"].T + p["b4"], "lap": lh @ p["W4"].T}
    for k, v in dh.items():
        out[k] = v @ p["W4"].T
    return out


def loss_and_grad(flat, txy, target, t_scale):
    """MSE = mean over samples and both outputs of (u_hat - target)^2, and
    its gradient (flat) by backpropagation."""
    p = unflatten(flat)
    txy = np.asarray(txy, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    z = normalise(txy[:, 0], txy[:, 1], txy[:, 2], t_scale)
    n = z.shape[0]
    h1 = np.tanh(z @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    h3 = np.tanh(h2 @ p["W3"].T + p["b3"])
    out = h3 @ p["W4"].T + p["b4"]
    r = out - target
    loss = float(np.mean(r * r))
    d_out = 2.0 * r / (2 * n)
    g = {"W4": d_out.T @ h3, "b4": d_out.sum(0)}
    d3 = (d_out @ p["W4"]) * (1.0 - h3 * h3)
    g["W3"], g["b3"] = d3.T @ h2, d3.sum(0)
    d2 = (d3 @ p["W3"]) * (1.0 - h2 * h2)
    g["W2"], g["b2"] = d2.T @ h1, d2.sum(0)
    d1 = (d2 @ p["W2"]) * (1.0 - h1 * h1)
    g["W1"], g["b1"] = d1.T @ z, d1.sum(0)
    return loss, flatten(g)


def adam_step(flat, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return flat - lr * mhat / (np.sqrt(vhat) + eps), m, v
