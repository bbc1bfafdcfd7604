"""The control-variate network on the GPU against the FP64 oracle evaluated
with the same BF16 weights: forward-mode channels, the training gradient,
Adam, training progress, and the control-variate interface solve."""
import os

import numpy as np
import pytest

import oracle.mlp as M
import workloads as W
from parity import assert_parity

pytestmark = pytest.mark.gpu
THREADS = min(16, os.cpu_count() or 1)
T = W.CV_T_SCALE


def curved_params(seed=1):
    rng = np.random.default_rng(seed)
    return (W.mlp_init(seed) * 2.5 + 0.05 * rng.standard_normal(M.N_PARAMS)).astype(np.float32)


def cuda32(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def test_eval_matches_oracle(fk):
    import torch
    cv = fk.FkCv(curved_params(), T)
    _, bf = cv.params()
    assert np.array_equal(bf, M.bf16_round(curved_params()))
    rng = np.random.default_rng(0)
    n = 1000                                   # ragged: 15 full wavefronts and a partial one
    txy = np.stack([rng.uniform(0, T, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)], 1).astype(np.float32)
    print(f"[gpu] cv eval n={n}", flush=True)
    g = cv.eval(cuda32(txy))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    t64 = txy.astype(np.float64)
    fm = M.forward_mode(bf, t64[:, 0], t64[:, 1], t64[:, 2], T)
    for k, key in enumerate(("val", "dx", "dy", "dt", "lap")):
        scale = np.abs(fm[key]).max()
        err = np.abs(g[:, :, k] - fm[key]).max() / scale
        print(f"channel {key}: max rel err {err:.2e} (scale {scale:.3g})", flush=True)
        assert err < 2e-4, key
    cv.close()


@pytest.mark.parametrize("mode,bar", [("split", 2e-4), ("bf16", 2e-2)])
def test_eval_grad_matches_oracle(fk, mode, bar):
    """The martingale kernels' (x, y) gradient against the FP64 forward mode
    of the same BF16 weights (channel-wise max-norm relative error): hi + lo
    operands near FP32, BF16-rounded activations within the network bar."""
    import torch
    cv = fk.FkCv(curved_params(3), T, grad_precision=mode)
    _, bf = cv.params()
    rng = np.random.default_rng(5)
    n = 1000                                   # ragged: 15 full wavefronts and a partial one
    txy = np.stack([rng.uniform(0, T, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)], 1).astype(np.float32)
    print(f"[gpu] cv eval_grad {mode} n={n}", flush=True)
    g = cv.eval_grad(cuda32(txy))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    t64 = txy.astype(np.float64)
    fm = M.forward_mode(bf, t64[:, 0], t64[:, 1], t64[:, 2], T)
    errs = []
    for k, key in enumerate(("dx", "dy")):
        scale = np.abs(fm[key]).max()
        errs.append(np.abs(g[:, :, k] - fm[key]).max() / scale)
        print(f"{mode} channel {key}: max rel err {errs[-1]:.2e} (scale {scale:.3g})", flush=True)
    assert max(errs) < bar
    if mode == "bf16":
        assert max(errs) > 1e-4             # the rounding is really taken once
    cv.close()


def test_grad_matches_oracle(fk):
    import torch
    cv = fk.FkCv(curved_params(2), T)
    _, bf = cv.params()
    rng = np.random.default_rng(4)
    n = 700                                    # ragged last tile
    txy = np.stack([rng.uniform(0, T, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)], 1).astype(np.float32)
    target = np.stack([txy[:, 1] + 0.05 * np.sin(6 * txy[:, 2]), txy[:, 2] - 0.03 * txy[:, 0] / T], 1)
    g, loss = cv.grad(cuda32(txy), cuda32(target))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    ref_loss, ref = M.loss_and_grad(bf, txy.astype(np.float64), target.astype(np.float32).astype(np.float64), T)
    cos = float(g @ ref / (np.linalg.norm(g) * np.linalg.norm(ref)))
    rel = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
    print(f"grad cosine {cos:.6f}, rel err {rel:.2e}; loss {float(loss.item()):.6e} vs {ref_loss:.6e}", flush=True)
    assert cos >= 0.999 and rel <= 2e-2
    assert abs(float(loss.item()) - ref_loss) <= 1e-2 * ref_loss
    cv.close()


def test_adam_matches_oracle(fk):
    import torch
    p0 = curved_params(3)
    cv = fk.FkCv(p0, T)
    rng = np.random.default_rng(5)
    p, m, v = p0.astype(np.float64), np.zeros(M.N_PARAMS), np.zeros(M.N_PARAMS)
    for step in range(1, 11):
        grad = (rng.standard_normal(M.N_PARAMS) * 1e-2).astype(np.float32)
        cv.adam_apply(cuda32(grad), 1e-3)
        p, m, v = M.adam_step(p, grad.astype(np.float64), m, v, step, 1e-3)
    torch.cuda.synchronize()
    master, bf = cv.params()
    assert np.abs(master - p).max() <= 1e-6 * max(1.0, np.abs(p).max())
    assert np.array_equal(bf, M.bf16_round(master))
    cv.close()


def test_training_reduces_loss(fk):
    import torch
    cv = fk.FkCv(W.mlp_init(0), T)
    rng = np.random.default_rng(6)
    n = 20000
    txy = np.stack([rng.uniform(0, T, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)], 1).astype(np.float32)
    target = np.stack([txy[:, 1] + 0.05 * np.sin(np.pi * txy[:, 1]) * np.sin(np.pi * txy[:, 2]),
                       txy[:, 2] - 0.04 * np.sin(np.pi * txy[:, 1]) * txy[:, 0] / T], 1).astype(np.float32)
    loss = cv.train(cuda32(txy), cuda32(target), steps=600, batch=2048, lr=3e-3, seed=1)
    torch.cuda.synchronize()
    loss = loss.cpu().numpy()
    print(f"training loss {loss[0]:.3e} -> {loss[-1]:.3e}", flush=True)
    assert np.all(np.isfinite(loss)) and loss[-20:].mean() < 0.05 * loss[:5].mean()
    # the trained network, evaluated in FP64 by the oracle, fits the targets
    _, bf = cv.params()
    fit = M.forward(bf, *txy.astype(np.float64).T, T)
    assert np.sqrt(np.mean((fit - target) ** 2)) < 0.02
    cv.close()


def test_training_graph_replays_and_matches_step_by_step(fk, oracle_mod):
    """fk_cv_train runs its loop as a captured graph that reads each call's
    values from device memory: two calls of 3 steps (the second a replay)
    give bitwise the weights of one call of 6, and both match a step-by-step
    reference built from the parity hooks -- the minibatch indices from the
    oracle's own Philox (counter (j, step, 0, 2) modulo n), the gradient of
    each minibatch (fk_cv_grad) and one Adam step (fk_cv_adam_apply)."""
    import torch
    rng = np.random.default_rng(8)
    n, batch, seed, lr = 5000, 300, 11, 2e-3
    txy = np.stack([rng.uniform(0, T, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)], 1).astype(np.float32)
    target = np.stack([txy[:, 1] + 0.03 * np.sin(5 * txy[:, 2]), txy[:, 2] - 0.02 * txy[:, 0] / T], 1)
    tg, tt = cuda32(txy), cuda32(target)
    a = fk.FkCv(curved_params(5), T)
    la = [a.train(tg, tt, steps=3, batch=batch, lr=lr, seed=seed) for _ in range(2)]
    b = fk.FkCv(curved_params(5), T)
    lb = b.train(tg, tt, steps=6, batch=batch, lr=lr, seed=seed)
    torch.cuda.synchronize()
    ma, _ = a.params()
    mb, _ = b.params()
    assert np.array_equal(ma, mb)
    assert np.array_equal(torch.cat(la).cpu().numpy(), lb.cpu().numpy())
    c = fk.FkCv(curved_params(5), T)
    for step in range(1, 7):
        ctr = np.stack([np.arange(batch), np.full(batch, step), np.zeros(batch), np.full(batch, 2)], 1)
        key = np.tile([seed & 0xffffffff, seed >> 32], (batch, 1))
        idx = (oracle_mod.philox(ctr, key)[:, 0] % n).astype(np.int64)
        g, _ = c.grad(cuda32(txy[idx]), cuda32(target[idx]))
        c.adam_apply(g, lr)
    torch.cuda.synchronize()
    mc, _ = c.params()
    err = np.abs(mc - mb).max() / np.abs(mb).max()
    print(f"graph-replayed training vs step by step: max rel diff {err:.2e}", flush=True)
    assert err < 1e-5
    for h in (a, b, c):
        h.close()


@pytest.mark.parametrize("stride", [2, 6])
def test_cv_solve_against_oracle(fk, oracle_mod, stride):
    import torch
    params = W.mlp_init(7)          # initial-scale network: moderate derivatives
    cv = fk.FkCv(params, T)
    _, bf = cv.params()
    dens = W.moving_bump()
    pts = W.interface_nodes(4, 4, 16)[::3]
    t, dt, N = 0.01, 1e-4, 256
    print(f"[gpu] cv solve stride={stride} nodes={len(pts)} N={N}", flush=True)
    g = fk.fk_interface_solve_cv(dens, W.Data(), pts, t, dt, N, cv, stride=stride, seed=3, exit_step=True,
                                 cv_scores=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}
    o = oracle_mod.fk_solve_cv(dens, W.Data(), pts, t, dt, N, seed=3, uhat=oracle_mod.UHAT_MLP, flat=bf,
                               t_scale=T, stride=stride, want_scores=True, want_exit=True, threads=THREADS)
    # plain part: the same paths as the plain solver, to the plain contract
    plain = {"xi": g["plain_xi"], "eta": g["plain_eta"], "se_xi": g["plain_se_xi"], "se_eta": g["plain_se_eta"],
             "exit_step": g["exit_step"]}
    po = {"mean": o["plain_mean"], "se": o["plain_se"], "exit_step": o["exit_step"]}
    assert_parity(plain, po, pts, label="plain part:")
    # CV part: per-path scores and node estimates
    same = g["exit_step"] == o["exit_step"]
    ds = np.abs(g["cv_scores"].astype(np.float64) - o["cv_scores"])[same]
    mean_g = np.stack([g["xi"], g["eta"]], 1)
    d = np.abs(mean_g - o["mean"])
    # The GPU network carries ~1e-5 relative error (split BF16 on MFMA,
    # FP32 accumulation), so a score sum(r ds) of size S is good to ~1e-5 S.
    smax = np.abs(o["cv_scores"]).max()
    print(f"cv: max |score diff| {ds.max():.2e} (max |score| {smax:.3g}), max |mean diff| {d.max():.2e}, "
          f"se ratio cv/plain {np.median(o['se'] / o['plain_se']):.3f}", flush=True)
    assert ds.max() < 2e-5 * max(1.0, smax)
    assert np.all(d <= 3 * o["se"]) and np.all(d <= 1e-5 * max(1.0, smax))
    cv.close()


@pytest.mark.parametrize("form", ["dynkin", "martingale"])
def test_cv_plans_change_only_the_schedule(fk, form):
    """Few paths per node on a long horizon: the default plan of the
    control-variate forms takes grabs of 32 to 128 paths by the node and
    path counts; every grab size, block size and node tile gives bitwise the
    same estimates, per-path scores and exit steps (each path draws from its
    own counters, and the estimator's sums are exact integers)."""
    import torch
    cv = fk.FkCv(W.mlp_init(7), T, identity_base=True)
    dens = W.moving_bump()
    pts = W.interface_nodes(4, 4, 16)[::2]
    t, dt, N = 0.01, 1e-4, 163                 # 100 steps: the long-horizon default
    fm = fk.FK_CV_DYNKIN if form == "dynkin" else fk.FK_CV_MARTINGALE
    print(f"[gpu] cv plans form={form} nodes={len(pts)} N={N}", flush=True)
    runs = []
    for plan in (None, {"chunk": 128}, {"chunk": 64}, {"chunk": 32}, {"chunk": 7, "block": 64},
                 {"chunk": 32, "node_tile": 4}):
        g = fk.fk_interface_solve_cv(dens, W.Data(), pts, t, dt, N, cv, stride=10, seed=3, form=fm, exit_step=True,
                                     cv_scores=True, plan=plan)
        torch.cuda.synchronize()
        runs.append({k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")})
    cv.close()
    for r in runs[1:]:
        for k in ("xi", "eta", "se_xi", "se_eta", "plain_xi", "plain_eta", "exit_step", "cv_scores", "total_steps"):
            assert np.array_equal(r[k], runs[0][k]), k


def test_trained_network_gain(fk):
    """What the trained network buys on the moving-bump workload: labels from
    plain Monte Carlo (132 time levels in [0, 0.1] x 1521 nodes x 1024
    paths), the default training schedule on the GPU (an identity-base
    network: u_hat = (x, y) + MLP), then control-variate solves at t = 0.1 on
    every 8th node, judged against the finite-difference reference, against
    plain Monte Carlo on the same paths, and against the linear control (the
    identity map's gradient, no network) on the same paths.  Away from the
    bump the solution's gradient is close to the identity, so the linear
    control alone already removes ~96% of the variance; the trained network
    must remove most of what is left: in the martingale form with the BF16
    gradient its variance is held below 0.3 of the linear control's at
    stride 20 and below 0.6 at stride 100 (measured: 0.10 and 0.28), and in
    the Dynkin form, whose integrand vanishes where u_hat solves the PDE,
    below 0.2 at stride 20 (measured: 0.052)."""
    import torch
    from paper_1402_0266_amd import cv_pipeline as P
    wl = W.MOVING_BUMP_1521
    nodes = wl.nodes()
    print("[gpu] cv gain: labels, training, solves", flush=True)
    txy, target = P.make_labels(wl.density, wl.data, nodes, W.cv_label_levels(132, W.CV_T_SCALE), wl.dt, 1024,
                                seed=1)
    cv = fk.FkCv(W.mlp_init(0), T, identity_base=True, grad_precision="bf16")
    loss = P.train_schedule(cv, txy, target, P.TRAIN_SCHEDULE, batch=8192, seed=2)
    assert loss.shape[0] == sum(n for n, _ in P.TRAIN_SCHEDULE)
    sub = np.arange(0, len(nodes), 8)
    fd = np.loadtxt(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"{wl.name}_fd.txt"))[sub]
    ref = fd[:, 2:4]
    assert np.abs(fd[:, :2] - nodes[sub]).max() < 1e-12

    def pair(r, a, b):
        return np.stack([r[a].cpu().numpy(), r[b].cpu().numpy()], 1)

    runs = {}
    for name, form, stride in (("martingale 20", fk.FK_CV_MARTINGALE, 20), ("martingale 100", fk.FK_CV_MARTINGALE, 100),
                               ("dynkin 20", fk.FK_CV_DYNKIN, 20)):
        g = fk.fk_interface_solve_cv(wl.density, wl.data, nodes[sub], wl.t, wl.dt, 2048, cv, stride=stride, seed=3,
                                     form=form)
        torch.cuda.synchronize()
        runs[name] = (pair(g, "xi", "eta"), pair(g, "se_xi", "se_eta"), pair(g, "plain_xi", "plain_eta"),
                      pair(g, "plain_se_xi", "plain_se_eta"))
    cv.close()
    loss = loss.cpu().numpy()
    # the linear control on the same paths: the identity data posed as a
    # 256-cell identity grid scored past the edge (the same scores), whose
    # bilinear gradient is exactly I
    import dataclasses
    G = 256
    x = torch.arange(G + 1, dtype=torch.float64, device="cuda") / G
    grids = (x.repeat(G + 1, 1).contiguous().view(-1), x[:, None].repeat(1, G + 1).contiguous().view(-1))
    gdata = dataclasses.replace(wl.data, init_kind=W.DATA_GRID, score_mode=W.SCORE_EXTEND)
    lin = fk.fk_interface_solve_cv(wl.density, gdata, nodes[sub], wl.t, wl.dt, 2048, None, stride=1 << 20, seed=3,
                                   form=fk.FK_CV_MARTINGALE_GRID, grids=grids)
    torch.cuda.synchronize()
    lps, lcs = pair(lin, "plain_se_xi", "plain_se_eta"), pair(lin, "se_xi", "se_eta")
    ratio_lin = float(np.mean(lcs ** 2) / np.mean(lps ** 2))
    print(f"loss {loss[0]:.3e} -> {loss[-200:].mean():.3e}; linear control: variance ratio to plain "
          f"{ratio_lin:.4f}", flush=True)
    bound = {"martingale 20": 0.3, "martingale 100": 0.6, "dynkin 20": 0.2}
    for name, (cvm, cvs, plm, pls) in runs.items():
        # the same paths as the linear control's (its bilinear identity equals x to rounding)
        assert np.allclose(lps, pls, rtol=1e-5, atol=0)
        rms_cv = float(np.sqrt(np.mean((cvm - ref) ** 2)))
        rms_pl = float(np.sqrt(np.mean((plm - ref) ** 2)))
        ratio = float(np.mean(cvs ** 2) / np.mean(pls ** 2))
        print(f"{name}: variance ratio to plain {ratio:.4f}, network / linear {ratio / ratio_lin:.3f}; "
              f"RMS vs FD: cv {rms_cv:.2e}, plain {rms_pl:.2e}", flush=True)
        assert ratio < bound[name] * ratio_lin
        assert rms_cv < 0.6 * rms_pl
        # the control-variate estimate is unbiased: within its error of the FD reference
        z = (cvm - ref) / np.sqrt(cvs ** 2 + fd[:, 4:6] ** 2)
        assert abs(float(z.mean())) < 0.5 and float(np.sqrt(np.mean(z ** 2))) < 1.5


@pytest.mark.parametrize("stride", [2, 20])
def test_cv_martingale_against_oracle(fk, oracle_mod, stride):
    """Martingale form: the same paths; the GPU takes the network's gradient
    with BF16 activations (relative error ~1e-2), which changes each path's
    martingale sum a little but not its zero mean."""
    import torch
    cv = fk.FkCv(W.mlp_init(7), T)
    _, bf = cv.params()
    dens = W.moving_bump()
    pts = W.interface_nodes(4, 4, 16)[::3]
    t, dt, N = 0.01, 1e-4, 512
    print(f"[gpu] cv martingale stride={stride} nodes={len(pts)} N={N}", flush=True)
    g = fk.fk_interface_solve_cv(dens, W.Data(), pts, t, dt, N, cv, stride=stride, seed=3, form=fk.FK_CV_MARTINGALE,
                                 exit_step=True, cv_scores=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}
    o = oracle_mod.fk_solve_cv(dens, W.Data(), pts, t, dt, N, seed=3, uhat=oracle_mod.UHAT_MLP, flat=bf, t_scale=T,
                               stride=stride, form=oracle_mod.CV_MARTINGALE, want_scores=True, want_exit=True,
                               threads=THREADS)
    plain = {"xi": g["plain_xi"], "eta": g["plain_eta"], "se_xi": g["plain_se_xi"], "se_eta": g["plain_se_eta"],
             "exit_step": g["exit_step"]}
    assert_parity(plain, {"mean": o["plain_mean"], "se": o["plain_se"], "exit_step": o["exit_step"]}, pts,
                  label="plain part:")
    same = g["exit_step"] == o["exit_step"]
    po = oracle_mod.fk_solve(dens, W.Data(), pts, t, dt, N, seed=3, want_scores=True, threads=THREADS)["scores"]
    msum = np.abs(po - o["cv_scores"])[same]           # |martingale sum| per path (oracle)
    ds = np.abs(g["cv_scores"].astype(np.float64) - o["cv_scores"])[same]
    rel = ds.max(axis=-1) / np.maximum(msum.max(axis=-1), 1e-3)
    mean_g = np.stack([g["xi"], g["eta"]], 1)
    d = np.abs(mean_g - o["mean"])
    print(f"martingale: max |score diff| {ds.max():.2e} (max |sum| {msum.max():.3g}, max rel {rel.max():.2e}), "
          f"max |mean diff| {d.max():.2e}, se ratio cv/plain {np.median(o['se'] / o['plain_se']):.3f}", flush=True)
    assert rel.max() < 0.05
    assert np.all(d <= 3 * o["se"]) and np.all(d <= 1e-5)
    assert np.all(np.abs(np.stack([g["se_xi"], g["se_eta"]], 1) - o["se"]) <= 0.05 * o["se"])
    cv.close()


@pytest.mark.parametrize("stride", [2, 20])
def test_cv_martingale_bf16_gradient_against_oracle(fk, oracle_mod, stride):
    """Martingale form with the gradient from BF16-rounded activations: the
    estimator stays unbiased for any gradient fixed before the block's
    increments, so per-node means agree with the oracle's FP64-gradient
    estimate on the same paths within 3 SE; the plain part is unchanged and
    each path's martingale sum moves by at most the gradient's error."""
    import torch
    cv = fk.FkCv(W.mlp_init(7), T, grad_precision="bf16")
    _, bf = cv.params()
    dens = W.moving_bump()
    pts = W.interface_nodes(4, 4, 16)[::3]
    t, dt, N = 0.01, 1e-4, 512
    print(f"[gpu] cv martingale bf16 stride={stride} nodes={len(pts)} N={N}", flush=True)
    g = fk.fk_interface_solve_cv(dens, W.Data(), pts, t, dt, N, cv, stride=stride, seed=3, form=fk.FK_CV_MARTINGALE,
                                 exit_step=True, cv_scores=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}
    o = oracle_mod.fk_solve_cv(dens, W.Data(), pts, t, dt, N, seed=3, uhat=oracle_mod.UHAT_MLP, flat=bf, t_scale=T,
                               stride=stride, form=oracle_mod.CV_MARTINGALE, want_scores=True, want_exit=True,
                               threads=THREADS)
    plain = {"xi": g["plain_xi"], "eta": g["plain_eta"], "se_xi": g["plain_se_xi"], "se_eta": g["plain_se_eta"],
             "exit_step": g["exit_step"]}
    assert_parity(plain, {"mean": o["plain_mean"], "se": o["plain_se"], "exit_step": o["exit_step"]}, pts,
                  label="plain part:")
    same = g["exit_step"] == o["exit_step"]
    po = oracle_mod.fk_solve(dens, W.Data(), pts, t, dt, N, seed=3, want_scores=True, threads=THREADS)["scores"]
    msum = np.abs(po - o["cv_scores"])[same]
    ds = np.abs(g["cv_scores"].astype(np.float64) - o["cv_scores"])[same]
    mean_g = np.stack([g["xi"], g["eta"]], 1)
    se_g = np.stack([g["se_xi"], g["se_eta"]], 1)
    d = np.abs(mean_g - o["mean"])
    print(f"martingale bf16: max |score diff| {ds.max():.2e} (largest |martingale sum| {msum.max():.3g}), "
          f"max |mean diff| {d.max():.2e} = {np.max(d / o['se']):.2f} se, se ratio gpu/oracle "
          f"{np.median(se_g / o['se']):.3f}", flush=True)
    # a 2e-2 relative gradient error moves a path's sum by at most that
    # fraction of the sums' scale (sums that cancel to ~0 have no scale of their own)
    assert ds.max() <= 2e-2 * msum.max()
    assert np.all(d <= 3 * o["se"])
    assert np.all(np.abs(se_g - o["se"]) <= 0.1 * o["se"])
    cv.close()


@pytest.mark.parametrize("stride", [2, 20])
def test_cv_grid_control_against_oracle(fk, oracle_mod, stride):
    """Martingale form with the grid initial data's gradient as the control
    (no network): a deformed mesh under two frozen bumps, exits scored with
    the grid continued past the edge, one mesh step."""
    import torch
    n = 48
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x)
    gx = X + 0.02 * np.sin(np.pi * X) * np.sin(2 * np.pi * Y)
    gy = Y + 0.015 * np.sin(2 * np.pi * X) * np.sin(np.pi * Y)
    dens = W.two_bumps(W.TIME_FROZEN, 0.0375)
    data = W.Data(init_kind=W.DATA_GRID, score_mode=W.SCORE_EXTEND, t_init=0.0375, grid_xi=gx.ravel(),
                  grid_eta=gy.ravel())
    nodes = W.interface_nodes(4, 4, 48)
    pts = np.concatenate([nodes[::7], nodes[np.minimum(nodes, 1 - nodes).min(1) < 0.05][::3]])
    t, dt, N = 5e-4, 2.5e-5, 2048
    grids = (torch.tensor(gx.ravel(), device="cuda"), torch.tensor(gy.ravel(), device="cuda"))
    print(f"[gpu] cv grid control stride={stride} nodes={len(pts)} N={N}", flush=True)
    g = fk.fk_interface_solve_cv(dens, data, pts, t, dt, N, None, stride=stride, seed=5, level_id=2,
                                 form=fk.FK_CV_MARTINGALE_GRID, exit_step=True, cv_scores=True, grids=grids)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}
    o = oracle_mod.fk_solve_cv(dens, data, pts, t, dt, N, seed=5, level_id=2, uhat=oracle_mod.UHAT_GRID,
                               stride=stride, form=oracle_mod.CV_MARTINGALE, want_scores=True, want_exit=True,
                               threads=THREADS)
    plain = {"xi": g["plain_xi"], "eta": g["plain_eta"], "se_xi": g["plain_se_xi"], "se_eta": g["plain_se_eta"],
             "exit_step": g["exit_step"]}
    assert_parity(plain, {"mean": o["plain_mean"], "se": o["plain_se"], "exit_step": o["exit_step"]}, pts,
                  shifted=False, label="plain part:")
    same = g["exit_step"] == o["exit_step"]
    ds = np.abs(g["cv_scores"].astype(np.float64) - o["cv_scores"])[same]
    d = np.abs(np.stack([g["xi"], g["eta"]], 1) - o["mean"])
    ratio = np.median(o["se"] / o["plain_se"])
    print(f"grid control: max |score diff| {ds.max():.2e}, max |mean diff| {d.max():.2e}, se cv/plain {ratio:.3f}",
          flush=True)
    # The bilinear gradient jumps across cell edges: where FP32 and FP64
    # positions sit on opposite sides of one, the path's G differs by that
    # jump times its block's Brownian part; like exit steps, such paths are
    # rare (99.9% agree to 1e-6) and their differences bounded.
    assert np.mean(ds.max(axis=-1) < 1e-6) >= 0.999 and ds.max() < 1e-3
    assert np.all(d <= 3 * o["se"]) and np.all(d <= 1e-5)
    assert np.all(np.abs(np.stack([g["se_xi"], g["se_eta"]], 1) - o["se"]) <= 0.01 * o["se"] + 1e-9)
    assert ratio < (0.1 if stride == 2 else 0.5)
    # a workspace of the plain size (its own CV records leave no room for
    # the per-cell gradient table): the kernel reads the grids instead, with
    # bitwise the same results
    small = torch.empty(fk.library().fk_interface_cv_workspace_bytes(len(pts), N), dtype=torch.uint8, device="cuda")
    h = fk.fk_interface_solve_cv(dens, data, pts, t, dt, N, None, stride=stride, seed=5, level_id=2,
                                 form=fk.FK_CV_MARTINGALE_GRID, exit_step=True, grids=grids, workspace=small,
                                 grad_table=False)
    torch.cuda.synchronize()
    assert h["_workspace"] is small
    for k in ("xi", "eta", "se_xi", "se_eta", "exit_step"):
        assert np.array_equal(h[k].cpu().numpy(), g[k]), k
    # a device mask: bitwise the full solve at its nodes, the rest untouched
    mask = np.arange(len(pts)) % 3 == 1
    sentinel = {k: torch.full(v.shape, 7, dtype=torch.float64 if v.dtype == np.float64 else
                              (torch.int32 if v.dtype == np.int32 else torch.float32), device="cuda")
                for k, v in g.items() if k != "total_steps"}
    m = fk.fk_interface_solve_cv(dens, data, torch.tensor(pts, device="cuda"), t, dt, N, None, stride=stride,
                                 seed=5, level_id=2, form=fk.FK_CV_MARTINGALE_GRID, exit_step=True, cv_scores=True,
                                 grids=grids, out=sentinel, mask=torch.tensor(mask.astype(np.uint8), device="cuda"))
    torch.cuda.synchronize()
    for k, v in g.items():
        if k == "total_steps":
            continue
        got = m[k].cpu().numpy()
        assert np.array_equal(got[mask], v[mask]), k
        assert np.all(got[~mask] == 7), k


@pytest.mark.parametrize("stride", [2, 20])
def test_cv_grid_base_against_oracle(fk, oracle_mod, stride):
    """Martingale form with the network as the deviation from the mesh
    (u_hat = bilinear grid initial data + network): a deformed mesh under two
    frozen bumps, one mesh step; the same paths as the oracle's with the same
    BF16 weights."""
    import torch
    n = 48
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x)
    gx = X + 0.02 * np.sin(np.pi * X) * np.sin(2 * np.pi * Y)
    gy = Y + 0.015 * np.sin(2 * np.pi * X) * np.sin(np.pi * Y)
    dens = W.two_bumps(W.TIME_FROZEN, 0.0375)
    data = W.Data(init_kind=W.DATA_GRID, score_mode=W.SCORE_EXTEND, t_init=0.0375, grid_xi=gx.ravel(),
                  grid_eta=gy.ravel())
    nodes = W.interface_nodes(4, 4, 48)
    pts = np.concatenate([nodes[::7], nodes[np.minimum(nodes, 1 - nodes).min(1) < 0.05][::3]])
    t, dt, N = 5e-4, 2.5e-5, 2048
    cv = fk.FkCv(W.mlp_init(7) * 0.2, T, base="grid")
    _, bf = cv.params()
    grids = (torch.tensor(gx.ravel(), device="cuda"), torch.tensor(gy.ravel(), device="cuda"))
    print(f"[gpu] cv grid base stride={stride} nodes={len(pts)} N={N}", flush=True)
    g = fk.fk_interface_solve_cv(dens, data, pts, t, dt, N, cv, stride=stride, seed=5, level_id=2,
                                 form=fk.FK_CV_MARTINGALE, exit_step=True, cv_scores=True, grids=grids)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}
    o = oracle_mod.fk_solve_cv(dens, data, pts, t, dt, N, seed=5, level_id=2, uhat=oracle_mod.UHAT_GRID_MLP, flat=bf,
                               t_scale=T, stride=stride, form=oracle_mod.CV_MARTINGALE, want_scores=True,
                               want_exit=True, threads=THREADS)
    plain = {"xi": g["plain_xi"], "eta": g["plain_eta"], "se_xi": g["plain_se_xi"], "se_eta": g["plain_se_eta"],
             "exit_step": g["exit_step"]}
    assert_parity(plain, {"mean": o["plain_mean"], "se": o["plain_se"], "exit_step": o["exit_step"]}, pts,
                  shifted=False, label="plain part:")
    same = g["exit_step"] == o["exit_step"]
    po = oracle_mod.fk_solve(dens, data, pts, t, dt, N, seed=5, level_id=2, want_scores=True,
                             threads=THREADS)["scores"]
    msum = np.abs(po - o["cv_scores"])[same]
    ds = np.abs(g["cv_scores"].astype(np.float64) - o["cv_scores"])[same]
    rel = ds.max(axis=-1) / np.maximum(msum.max(axis=-1), 1e-3)
    d = np.abs(np.stack([g["xi"], g["eta"]], 1) - o["mean"])
    ratio = np.median(o["se"] / o["plain_se"])
    print(f"grid base: max |score diff| {ds.max():.2e}, max rel {rel.max():.2e}, max |mean diff| {d.max():.2e}, "
          f"se cv/plain {ratio:.3f}", flush=True)
    # as for the grid control, a path whose FP32 and FP64 positions sit on
    # opposite sides of a cell edge takes a different mesh gradient: rare
    assert np.mean(rel < 0.05) >= 0.999 and ds.max() < 1e-3
    assert np.all(d <= 3 * o["se"] + 1e-7) and np.all(d <= 1e-5)
    assert np.all(np.abs(np.stack([g["se_xi"], g["se_eta"]], 1) - o["se"]) <= 0.05 * o["se"] + 1e-9)
    # the Dynkin form has no grid base
    with pytest.raises(fk.FkError):
        fk.fk_interface_solve_cv(dens, data, pts, t, dt, 16, cv, stride=stride, form=fk.FK_CV_DYNKIN, grids=grids)
    cv.close()


def test_identity_base_eval_and_grad(fk):
    """The identity base: every evaluation adds (x, y) and the identity to the
    network's values and gradients, and training fits target - (x, y)."""
    import torch
    cv = fk.FkCv(curved_params(3), T, identity_base=True)
    _, bf = cv.params()
    rng = np.random.default_rng(5)
    n = 777
    txy = np.stack([rng.uniform(0, T, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n)], 1).astype(np.float32)
    print(f"[gpu] cv identity base eval n={n}", flush=True)
    g = cv.eval(cuda32(txy))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    t64 = txy.astype(np.float64)
    fm = M.forward_mode(bf, t64[:, 0], t64[:, 1], t64[:, 2], T)
    fm["val"] = fm["val"] + t64[:, 1:3]
    fm["dx"] = fm["dx"] + np.array([1.0, 0.0])
    fm["dy"] = fm["dy"] + np.array([0.0, 1.0])
    for k, key in enumerate(("val", "dx", "dy", "dt", "lap")):
        scale = np.abs(fm[key]).max()
        err = np.abs(g[:, :, k] - fm[key]).max() / scale
        print(f"channel {key}: max rel err {err:.2e} (scale {scale:.3g})", flush=True)
        assert err < 2e-4, key
    target = np.stack([txy[:, 1] + 0.05 * np.sin(6 * txy[:, 2]), txy[:, 2] - 0.03 * txy[:, 0] / T], 1)
    gg, loss = cv.grad(cuda32(txy), cuda32(target))
    torch.cuda.synchronize()
    gg = gg.cpu().numpy().astype(np.float64)
    resid = target.astype(np.float32).astype(np.float64) - t64[:, 1:3]
    ref_loss, ref = M.loss_and_grad(bf, t64, resid, T)
    cos = float(gg @ ref / (np.linalg.norm(gg) * np.linalg.norm(ref)))
    print(f"base grad cosine {cos:.6f}; loss {float(loss.item()):.6e} vs {ref_loss:.6e}", flush=True)
    assert cos >= 0.999 and abs(float(loss.item()) - ref_loss) <= 1e-2 * ref_loss
    cv.close()


@pytest.mark.parametrize("form", ["dynkin", "martingale"])
def test_identity_base_solve_against_oracle(fk, oracle_mod, form):
    import torch
    cv = fk.FkCv(W.mlp_init(7), T, identity_base=True)
    _, bf = cv.params()
    dens = W.moving_bump()
    pts = W.interface_nodes(4, 4, 16)[::3]
    t, dt, N, stride = 0.01, 1e-4, 512, 6
    f_gpu = fk.FK_CV_DYNKIN if form == "dynkin" else fk.FK_CV_MARTINGALE
    f_or = oracle_mod.CV_DYNKIN if form == "dynkin" else oracle_mod.CV_MARTINGALE
    print(f"[gpu] cv identity base {form} nodes={len(pts)} N={N}", flush=True)
    g = fk.fk_interface_solve_cv(dens, W.Data(), pts, t, dt, N, cv, stride=stride, seed=3, form=f_gpu,
                                 exit_step=True, cv_scores=True)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in g.items() if not k.startswith("_")}
    o = oracle_mod.fk_solve_cv(dens, W.Data(), pts, t, dt, N, seed=3, uhat=oracle_mod.UHAT_MLP_BASE, flat=bf,
                               t_scale=T, stride=stride, form=f_or, want_scores=True, want_exit=True, threads=THREADS)
    same = g["exit_step"] == o["exit_step"]
    assert np.mean(same) >= 0.999
    ds = np.abs(g["cv_scores"].astype(np.float64) - o["cv_scores"])[same]
    smax = np.abs(o["cv_scores"]).max()
    d = np.abs(np.stack([g["xi"], g["eta"]], 1) - o["mean"])
    print(f"{form} with base: max |score diff| {ds.max():.2e} (max |score| {smax:.3g}), max |mean diff| {d.max():.2e}, "
          f"se ratio cv/plain {np.median(o['se'] / o['plain_se']):.3f}", flush=True)
    assert ds.max() < 2e-5 * max(1.0, smax)
    assert np.all(d <= 3 * o["se"]) and np.all(d <= 1e-5 * max(1.0, smax))
    cv.close()
