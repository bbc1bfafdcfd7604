"""Benchmark of the Monte-Carlo interface solve on one MI355X.

Workload: the moving-bump interface problem -- 4x4 sub-domains of the unit
square, 3 vertical + 3 horizontal interface lines with 255 nodes each (1521
unique nodes), w = 1 + 20 exp(-|X - c(tau)|^2 / 0.005) with the centre
c(tau) = (1/2 + cos(2 pi tau)/4, 1/2 + sin(2 pi tau)/4), t = 0.1, dt = 1e-5,
FP32 paths, FP64 estimator.  Inputs are synthetic and generated on the host.

Metric: interface nodes/s at RMS error 1e-3 against the finite-difference
reference (stored under tests/golden, written from the CPU oracle).  A pilot
solve at the configured 10^5 paths/node gives the mean per-node score variance
s2 and the bias b^2 = max(0, RMS^2 - s2/N); the paths needed for RMS 1e-3 are
N* = ceil(s2 / (1e-6 - b^2)); each timed step is one full solve at N*.

The same line reports, as extra objects:

* "cv": the learned control variate on the same workload -- training labels
  from batched plain solves (132 time levels in [0, 0.1] x 1521 nodes x 1024
  paths), 16000 Adam steps on the GPU (a constant learning rate, then two
  decays), then the control-variate solve in the form (martingale with the
  hi + lo or the BF16 gradient, or Dynkin) and at the stride that reach RMS
  1e-3 fastest: pilots at 4096 paths give each candidate's N*, each
  candidate is timed once at its N*, and the fastest is timed.  The
  network fits the deviation from the identity map (u_hat = (x, y) + MLP);
  the same pipeline with the plain-output network, with the identity-base
  network fitted by 2000 Adam steps at lr 1e-3 only, and the identity's
  gradient alone as the control, are reported beside it.  Throughput is
  quoted for the solve alone and with the labels and training counted once.
* "bridge": the same workload with the Brownian-bridge exit test (bias and
  rate at RMS 1e-3) at dt = 1e-5 and at coarser steps, the discrete test
  beside it.
* "batched": 64 time levels t_k = 0.01 k of the moving bump with random
  2x2..8x8 layouts on G = 128 (66047 nodes), 2^16 paths per node, autotuned
  and captured in a HIP graph; one replay timed.
* "paper_run": the paper's own run (Sect. 5) -- the moving ring w = 1/rho
  on 41 x 41 nodes in 2 x 2 sub-domains, mesh step 1e-3 in 20 sub-steps,
  10^4 paths per simulated interface node, equidistributed edges,
  t <= 0.75; with the analytic drift, with the paper's data path (w sampled
  on the grid, finite-difference drift, bilinear between nodes), and with
  that data path and key points (the run as the paper describes it).
* "steady": the elliptic variant -- one-shot steady meshes of the static
  bump (64-cell grid) and of the paper's ring (41 x 41 grid), with the
  global steady solve beside them.
* "mesh_run": the time-dependent run -- 8 x 8 sub-domains on a 768-cell
  grid, two counter-rotating bumps, 200 mesh steps of 5e-4 with 20
  Euler-Maruyama steps each, 2^14 paths per interface node (10689 nodes),
  64 FP64 sub-domain solves per step; with the network refitted every 20
  steps, with the mesh's own gradient as the control, and plain; mesh
  quality is recorded every step (the tests compare it with the oracle's
  global step).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-cv] [--no-mesh-run]
                    [--no-batched] [--no-paper-run] [--no-bridge] [--no-steady]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

METRIC = "interface nodes/s at RMS err 1e-3 (plain MC vs MLP control variate), % FP32 peak"
FP32_PEAK_TFLOPS = 157.3
# FP32 operations of one Euler-Maruyama step of the moving-bump path, counted
# from the method (an FMA counts 2, a transcendental 1; the integer Philox work
# and the compensated position update are not counted):
#   Box-Muller 9  (2 uniform scalings, log, radius scale, sqrt, cos, sin, 2 products)
#   moving centre 9 (PDE time fma, angle, cos, sin, 2 radius products, 2 centre adds)
#   drift 14      (2 differences, r^2 mul+fma, exponent scale, exp, w = 1 + A e fma,
#                  2A/s2 e, reciprocal, product, 2 components)
#   Euler-Maruyama update 4 (2 fma)
FLOP_PER_STEP = 36
# The martingale form's network gradient on MFMA: value, d/dx and d/dy
# channels through the two 64 x 64 hidden products, 2 FLOP per
# multiply-add: 3 x 2 x 2 x 64 x 64 per evaluation point.
NET_GRAD_FLOP = 3 * 2 * 2 * 64 * 64
# The Dynkin form's five channels (value, d/dt, d/dx, d/dy, Laplacian)
# through the same two products.
NET_DYNKIN_FLOP = 5 * 2 * 2 * 64 * 64
BF16_PEAK_TFLOPS = 2500.0
# Paths per node of the control-variate kernels' profile with the grid
# full; the Dynkin kernel is also profiled at the timed solve's N*.
CV_PROFILE_PATHS = 2952

# HBM traffic of the path kernel from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
# (scaled by a plain 1 GiB copy: fetch x2.0, write x1.0) on the moving-bump
# solve at N* = 73920 (1521 x 578 chunks of 128 paths), per path, valid only
# for the kernel sources it was measured on (hash below); otherwise null.
TRAFFIC_BYTES_PER_PATH = (2.0 * 244.75 + 1.0 * 505266.5625) * 1024 / (1521 * 73920)
TRAFFIC_SOURCE_HASH = "ba5ecf16793f7980"
KERNEL_SOURCES = ["paper_1402_0266_amd/csrc/fk_paths.hip", "paper_1402_0266_amd/csrc/fk_device.hpp",
                  "paper_1402_0266_amd/csrc/fk_internal.hpp", "paper_1402_0266_amd/csrc/fk_pathstep.hpp",
                  "paper_1402_0266_amd/csrc/fk_accum.hpp"]


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_fd_reference(name: str):
    path = os.path.join(ROOT, "tests", "golden", f"{name}_fd.txt")
    if not os.path.exists(path):
        return None
    return np.loadtxt(path)


def rms_against(fd, xi, eta):
    ref = fd[:, 2:4]
    est = np.stack([xi, eta], 1)
    return float(np.sqrt(np.mean((est - ref) ** 2)))


def host_cores():
    """CPUs this process may run on: its affinity set, cut to the cgroup's CPU
    quota when one is set; with os.cpu_count() and the CPU model."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    try:
        quota, period = open("/sys/fs/cgroup/cpu.max").read().split()[:2]
        if quota != "max":
            n = max(1, min(n, int(int(quota) // int(period))))
    except (OSError, ValueError):
        pass
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return n, os.cpu_count() or 1, model


def cpu_baseline(wl, n_star, sample_nodes=96, sample_paths=2048):
    """The CPU oracle on a bounded sample: sample_nodes nodes spread evenly over the
    canonical order, sample_paths paths each, on every host core this process may
    use, scaled to nodes/s at N* paths per node."""
    import oracle
    oracle.build()
    threads, nproc, model = host_cores()
    pts = wl.nodes()
    sel = np.arange(0, len(pts), max(1, len(pts) // sample_nodes))[:sample_nodes]
    t0 = time.perf_counter()
    oracle.fk_solve(wl.density, wl.data, pts[sel], wl.t, wl.dt, sample_paths, wl.seed, node_ids=sel,
                    threads=threads)
    el = time.perf_counter() - t0
    nodes_per_s = len(sel) / el * (sample_paths / n_star)
    return {"value": nodes_per_s, "unit": "nodes/s", "cores": threads, "kind": "oracle",
            "nproc": nproc, "cpu_model": model, "build": "gcc -O3 -fopenmp",
            "sample": f"{len(sel)} nodes (every {len(pts) // sample_nodes}th) x {sample_paths} paths, "
                      f"{el:.2f}s, scaled by {sample_paths}/{n_star} paths"}


def _stack(r, keys):
    return np.stack([r[keys[0]].cpu().numpy(), r[keys[1]].cpu().numpy()], 1)


def measure_cv(fk, wl, pts, fd, steps, warmup, label_paths=1024, pilot_paths=4096, identity_base=False,
               schedule=None):
    """Labels, training (Adam stages of (steps, lr); the pipeline's default
    schedule if None) and the control-variate solve; nodes/s at RMS 1e-3."""
    import torch
    from paper_1402_0266_amd import cv_pipeline as P
    n_nodes = len(pts)
    ref = fd[:, 2:4]
    print("[bench] cv: labels", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    txy, target = P.make_labels(wl.density, wl.data, pts, W.cv_label_levels(132, W.CV_T_SCALE), wl.dt, label_paths,
                                seed=1)
    torch.cuda.synchronize()
    t_labels = time.perf_counter() - t0
    cv = fk.FkCv(W.mlp_init(0), W.CV_T_SCALE, identity_base=identity_base)
    pts = torch.tensor(pts, dtype=torch.float64, device="cuda")     # resident coordinates
    t0 = time.perf_counter()
    schedule = P.TRAIN_SCHEDULE if schedule is None else schedule
    loss = P.train_schedule(cv, txy, target, schedule, batch=8192, seed=2)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    loss = loss.cpu().numpy()

    def solve(n_paths, form, stride, plain=True):
        # plain=False: the control-variate estimates only (the plain estimate
        # on the same paths is a diagnostic and costs a second pass)
        return fk.fk_interface_solve_cv(wl.density, wl.data, pts, wl.t, wl.dt, n_paths, cv, stride=stride,
                                        seed=wl.seed, form=form, plain=plain)

    def pilot(form, stride, grad="split"):
        cv.set_grad_precision(grad)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = solve(pilot_paths, form, stride)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        est, se = _stack(r, ("xi", "eta")), _stack(r, ("se_xi", "se_eta"))
        var = float(np.mean(se ** 2) * pilot_paths)
        pse = _stack(r, ("plain_se_xi", "plain_se_eta"))
        b2 = max(0.0, float(np.mean((est - ref) ** 2)) - var / pilot_paths)
        n_star = int(math.ceil(var / (1e-6 - b2))) if b2 < 1e-6 else None
        return {"form": "martingale" if form == fk.FK_CV_MARTINGALE else "dynkin", "stride": stride,
                "grad": grad if form == fk.FK_CV_MARTINGALE else "split", "pilot_s": el, "var": var, "var_ratio": float(np.mean(pse ** 2) / np.mean(se ** 2)),
                "bias": math.sqrt(b2), "n_star": n_star,
                "predicted_s": None if n_star is None else el * n_star / pilot_paths}

    solve(256, fk.FK_CV_MARTINGALE, 20)         # first-launch costs out of the pilots
    solve(256, fk.FK_CV_DYNKIN, 20)
    pilots = ([pilot(fk.FK_CV_MARTINGALE, s) for s in (20, 100, 500, 2000)] +
              [pilot(fk.FK_CV_MARTINGALE, s, "bf16") for s in (20, 50, 100, 500)] +
              [pilot(fk.FK_CV_DYNKIN, s) for s in (20, 50, 100, 200, 500)])
    # Every candidate timed once at its own N*: below a few thousand paths
    # per node the grid is no longer full and the pilots' time does not
    # scale to N*.
    forms = {"martingale": fk.FK_CV_MARTINGALE, "dynkin": fk.FK_CV_DYNKIN}
    for p in pilots:
        if not p["n_star"]:
            continue
        cv.set_grad_precision(p["grad"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solve(max(2, p["n_star"]), forms[p["form"]], p["stride"], plain=False)
        torch.cuda.synchronize()
        p["s_at_n_star"] = time.perf_counter() - t0
    best = min((p for p in pilots if p["n_star"]), key=lambda p: p["s_at_n_star"])
    form, stride, n_star = forms[best["form"]], best["stride"], max(2, best["n_star"])
    cv.set_grad_precision(best["grad"])
    print(f"[bench] cv: {best['form']} stride {stride} ({best['grad']} gradient), N* = {n_star}", file=sys.stderr,
          flush=True)
    for _ in range(warmup):
        solve(n_star, form, stride, plain=False)
    torch.cuda.synchronize()
    fk.fk_timing_enable(True)
    kern = []
    t0 = time.perf_counter()
    for _ in range(steps):
        r = solve(n_star, form, stride, plain=False)
        kern.append(fk.fk_timing_last()[0])
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    fk.fk_timing_enable(False)
    rms = float(np.sqrt(np.mean((_stack(r, ("xi", "eta")) - ref) ** 2)))
    steps_cv = int(r["total_steps"].item())
    cv.close()
    # Beside the network: the same martingale estimator with the identity
    # map's gradient (the linear control, no training).  The identity data
    # posed as a 256-cell identity grid scored past the edge give the same
    # scores; its bilinear gradient is exactly I.
    import dataclasses
    G = 256
    x = torch.arange(G + 1, dtype=torch.float64, device="cuda") / G
    gx, gy = x.repeat(G + 1, 1).contiguous(), x[:, None].repeat(1, G + 1).contiguous()
    gdata = dataclasses.replace(wl.data, init_kind=W.DATA_GRID, score_mode=W.SCORE_EXTEND)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rl = fk.fk_interface_solve_cv(wl.density, gdata, pts, wl.t, wl.dt, pilot_paths, None, stride=1 << 20,
                                  seed=wl.seed, form=fk.FK_CV_MARTINGALE_GRID, grids=(gx.view(-1), gy.view(-1)))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    est, se = _stack(rl, ("xi", "eta")), _stack(rl, ("se_xi", "se_eta"))
    pse = _stack(rl, ("plain_se_xi", "plain_se_eta"))
    var = float(np.mean(se ** 2) * pilot_paths)
    b2 = max(0.0, float(np.mean((est - ref) ** 2)) - var / pilot_paths)
    n_lin = int(math.ceil(var / (1e-6 - b2))) if b2 < 1e-6 else None
    linear = {"form": "martingale, identity gradient", "pilot_s": el, "var": var,
              "var_ratio": float(np.mean(pse ** 2) / np.mean(se ** 2)), "bias": math.sqrt(b2), "n_star": n_lin,
              "predicted_nodes_per_s": None if n_lin is None else n_nodes / (el * n_lin / pilot_paths)}
    if n_lin:
        # and timed at its own N*, like the network's solve
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rl = fk.fk_interface_solve_cv(wl.density, gdata, pts, wl.t, wl.dt, max(2, n_lin), None, stride=1 << 20,
                                      seed=wl.seed, form=fk.FK_CV_MARTINGALE_GRID, grids=(gx.view(-1), gy.view(-1)),
                                      plain=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        linear.update({"paths_per_node": max(2, n_lin), "s_per_solve": el, "nodes_per_s": n_nodes / el,
                       "rms_err": float(np.sqrt(np.mean((_stack(rl, ("xi", "eta")) - ref) ** 2)))})
    kms = float(np.mean(kern))
    return {
        "form": best["form"], "stride": stride, "grad": best["grad"], "paths_per_node": n_star, "rms_err": rms,
        "s_per_solve": wall, "path_kernel_ms": kms,
        "roofline": cv_roofline(steps_cv, stride, kms, best["form"], best["grad"]),
        "nodes_per_s": n_nodes / wall,
        "nodes_per_s_incl_labels_and_training": n_nodes / (wall + t_labels + t_train),
        "labels": {"levels": 132, "paths": label_paths, "n": int(txy.shape[0]), "s": t_labels},
        "training": {"schedule": [list(x) for x in schedule], "batch": 8192, "s": t_train,
                     "loss_first": float(loss[0]),
                     "loss_last50": float(loss[-50:].mean())},
        "pilots": pilots,
        "linear_control": linear,
    }


def cv_roofline(path_steps, stride, kernel_ms, form, grad):
    """Roofline of the control-variate path kernel: FP32 VALU on the path
    steps (FLOP_PER_STEP each) against the FP32 vector peak, and the
    network's products on MFMA against the dense BF16 peak.  The network's
    algorithmic work is NET_GRAD_FLOP (martingale form) or NET_DYNKIN_FLOP
    (Dynkin form) per evaluation point, one evaluation per `stride` steps of
    a path (path_steps / stride); the hi + lo split issues each product
    twice, which counts as work done but not as algorithmic work."""
    fp32 = FLOP_PER_STEP * path_steps / (kernel_ms * 1e-3) / 1e12
    evals = path_steps / stride
    per_eval = NET_GRAD_FLOP if form == "martingale" else NET_DYNKIN_FLOP
    mf = per_eval * evals / (kernel_ms * 1e-3) / 1e12
    return {"kernel": "fk_mg_path_kernel" if form == "martingale" else "fk_cv_path_kernel", "bound": "alu",
            "achieved": fp32, "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": fp32 / FP32_PEAK_TFLOPS, "flop_per_path_step": FLOP_PER_STEP,
            "mfma": {"achieved": mf, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": mf / BF16_PEAK_TFLOPS,
                     "flop_per_eval": per_eval, "evals_per_launch": evals,
                     "issued_per_algorithmic": 2 if grad == "split" else 1}}


def measure_batched(fk, probe_paths=512):
    """64 time levels of the moving bump with random 2x2..8x8 layouts on
    G = 128 (66047 nodes), dt = 1e-5, 2^16 paths per node: autotuned plan,
    captured in a HIP graph, one replay timed."""
    import torch
    dens = W.moving_bump()
    lv = W.batched_levels(64, G=128)
    levels = [(dens, t, 0.0, pts, k) for k, (t, px, py, pts) in enumerate(lv, start=1)]
    n_paths, dt = 1 << 16, 1e-5
    b = fk.FkBatch(levels, W.Data(), dt, n_paths, seed=0)
    print(f"[bench] batched: {b.n_total} nodes, autotune at {probe_paths} paths", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = b.autotune(probe_paths)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    out = b.outputs()
    stream = torch.cuda.Stream()
    b.capture(out, stream)
    print(f"[bench] batched: replay with plan {plan}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.replay(stream)
    stream.synchronize()
    wall = time.perf_counter() - t0
    steps = int(out["total_steps"].item())
    b.close()
    return {"workload": "64 levels t_k = 0.01 k of the moving bump, random 2x2..8x8 layouts on G = 128, "
                        "dt = 1e-5, 2^16 paths/node, one graph-captured persistent launch",
            "levels": 64, "nodes": int(b.n_total), "paths_per_node": n_paths, "plan": plan,
            "autotune_s": t_tune, "s": wall, "nodes_per_s": b.n_total / wall,
            "path_steps": steps, "path_steps_per_s": steps / wall,
            "fp32_frac": FLOP_PER_STEP * steps / wall / 1e12 / FP32_PEAK_TFLOPS}


def measure_paper_run():
    """The paper's run (Sect. 5): the moving ring w = 1/rho on 41 x 41 nodes
    in 2 x 2 sub-domains, mesh step 1e-3 in 20 sub-steps, 10^4 paths per
    interface node (all 77), equidistributed edges, up to t = 0.75; with the
    analytic drift, and with the paper's data path (w sampled on the mesh
    grid at each step, drift by finite differences, bilinear)."""
    import torch
    from paper_1402_0266_amd.mesh_run import PAPER_RING_RUN, MeshRun, MeshRunConfig, paper_ring_density
    res = {"workload": "paper's run: ring w = 1/rho (alpha 10, beta -50), 41x41 nodes, 2x2 sub-domains, "
                       "dt_mesh 1e-3 / 20 sub-steps, 1e4 paths on all 77 interface nodes, t <= 0.75"}
    meshes = {}
    variants = (("analytic", {"density_data": "analytic"}), ("grid", {"density_data": "grid"}),
                ("grid_keys", {"density_data": "grid", "key_points": True}))
    for name, kw in variants:
        cfg = MeshRunConfig(**{**PAPER_RING_RUN, **kw})
        print(f"[bench] paper run ({name}): {cfg.n_steps} steps", file=sys.stderr, flush=True)
        run = MeshRun(cfg, density_fn=paper_ring_density)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run.run()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        q = run.qualities()
        _, se = run.interface_values()
        meshes[name] = run.mesh()
        run.close()
        snaps = {f"t={0.25 * k:.2f}": {"min_jac": float(q[250 * k - 1, 0]), "max_skew": float(q[250 * k - 1, 1])}
                 for k in (1, 2, 3)}
        res[name] = {"steps": cfg.n_steps, "s_total": wall, "ms_per_step": wall / cfg.n_steps * 1e3,
                     "min_jac_min": float(q[:, 0].min()), "max_skew_max": float(q[:, 1].max()),
                     "se_median": float(np.nanmedian(se)), "quality": snaps,
                     "simulated_nodes_mean": float(np.mean(run.n_keys)) if run.n_keys else float(run.n_nodes)}
    for name in ("grid", "grid_keys"):
        res[name]["final_mesh_max_diff_vs_analytic"] = float(
            max(np.abs(meshes["analytic"][c] - meshes[name][c]).max() for c in (0, 1)))
    return res


def cv_kernels_only(fk, n_paths=CV_PROFILE_PATHS):
    """The control-variate kernels, for the profiler: the Dynkin kernel at
    strides 100 and 200 at the timed solve's N* (163 and 289 paths per node)
    and at n_paths; the martingale kernel with the network at strides 500
    and 20, with the hi + lo and the BF16 gradient, and the linear control,
    at n_paths; two launches each.  The weights do not change the work: an
    untrained identity-base network."""
    import dataclasses

    import torch
    wl = W.MOVING_BUMP_1521
    pts = torch.tensor(wl.nodes(), dtype=torch.float64, device="cuda")
    cv = fk.FkCv(W.mlp_init(0), W.CV_T_SCALE, identity_base=True)
    cvb = fk.FkCv(W.mlp_init(0), W.CV_T_SCALE, identity_base=True, grad_precision="bf16")
    G = 256
    x = torch.arange(G + 1, dtype=torch.float64, device="cuda") / G
    grids = (x.repeat(G + 1, 1).contiguous().view(-1), x[:, None].repeat(1, G + 1).contiguous().view(-1))
    gdata = dataclasses.replace(wl.data, init_kind=W.DATA_GRID, score_mode=W.SCORE_EXTEND)
    res = {}
    fk.fk_timing_enable(True)
    def dynkin(n, stride):
        return lambda: fk.fk_interface_solve_cv(wl.density, wl.data, pts, wl.t, wl.dt, n, cv, stride=stride,
                                                seed=wl.seed, form=fk.FK_CV_DYNKIN, plain=False)

    for name, call in (
            ("dynkin_stride100_n163", dynkin(163, 100)),
            ("dynkin_stride200_n289", dynkin(289, 200)),
            ("dynkin_stride100", dynkin(n_paths, 100)),
            ("martingale_stride500", lambda: fk.fk_interface_solve_cv(wl.density, wl.data, pts, wl.t, wl.dt, n_paths,
                                                                      cv, stride=500, seed=wl.seed,
                                                                      form=fk.FK_CV_MARTINGALE, plain=False)),
            ("martingale_stride20", lambda: fk.fk_interface_solve_cv(wl.density, wl.data, pts, wl.t, wl.dt, n_paths,
                                                                     cv, stride=20, seed=wl.seed,
                                                                     form=fk.FK_CV_MARTINGALE, plain=False)),
            ("martingale_bf16_stride500", lambda: fk.fk_interface_solve_cv(wl.density, wl.data, pts, wl.t, wl.dt,
                                                                           n_paths, cvb, stride=500, seed=wl.seed,
                                                                           form=fk.FK_CV_MARTINGALE, plain=False)),
            ("martingale_bf16_stride20", lambda: fk.fk_interface_solve_cv(wl.density, wl.data, pts, wl.t, wl.dt,
                                                                          n_paths, cvb, stride=20, seed=wl.seed,
                                                                          form=fk.FK_CV_MARTINGALE, plain=False)),
            ("linear", lambda: fk.fk_interface_solve_cv(wl.density, gdata, pts, wl.t, wl.dt, n_paths, None,
                                                        stride=1 << 20, seed=wl.seed, form=fk.FK_CV_MARTINGALE_GRID,
                                                        plain=False, grids=grids))):
        ms, steps = [], []
        for _ in range(2):
            r = call()
            torch.cuda.synchronize()
            ms.append(fk.fk_timing_last()[0])
            steps.append(int(r["total_steps"].item()))
        res[name] = {"path_kernel_ms": ms, "path_steps": steps}
    fk.fk_timing_enable(False)
    cv.close()
    cvb.close()
    return {"cv_kernels": res, "n_paths": n_paths, "nodes": int(pts.shape[0])}


def measure_bridge(fk, wl, pts, fd, pilot_paths=100000):
    """The headline workload with the Brownian-bridge exit test and with
    exponential time-stepping, at the configured dt and at coarser steps
    (plain discrete test beside them): a pilot gives the variance and the
    bias against the FD reference, N* the paths for RMS 1e-3, and one timed
    solve at N* the rate."""
    import dataclasses

    import torch
    pts = torch.tensor(pts, dtype=torch.float64, device="cuda")     # resident coordinates
    res = []
    modes = {"discrete": wl.data.score_mode, "bridge": W.SCORE_BRIDGE, "exponential": W.SCORE_EXPONENTIAL}
    for dt, mode in ((1e-5, "bridge"), (4e-5, "discrete"), (4e-5, "bridge"), (4e-5, "exponential"),
                     (1e-4, "discrete"), (1e-4, "bridge"), (1e-4, "exponential"), (2.5e-4, "exponential")):
        bridge = mode == "bridge"
        data = dataclasses.replace(wl.data, score_mode=modes[mode])
        print(f"[bench] bridge leg: dt {dt:g}, {mode}", file=sys.stderr, flush=True)
        r = fk.fk_interface_solve(wl.density, data, pts, wl.t, dt, pilot_paths, wl.seed)
        est, se = _stack(r, ("xi", "eta")), _stack(r, ("se_xi", "se_eta"))
        var = float(np.mean(se ** 2) * pilot_paths)
        b2 = max(0.0, float(np.mean((est - fd[:, 2:4]) ** 2)) - var / pilot_paths)
        row = {"dt": dt, "mode": mode, "bridge": bridge, "var": var, "bias": math.sqrt(b2)}
        if b2 < 0.9e-6:
            n_star = int(math.ceil(var / (1e-6 - b2)))
            fk.fk_timing_enable(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fk.fk_interface_solve(wl.density, data, pts, wl.t, dt, n_star, wl.seed)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            kms, _ = fk.fk_timing_last()
            fk.fk_timing_enable(False)
            est = _stack(r, ("xi", "eta"))
            row.update({"n_star": n_star, "s_per_solve": wall, "path_kernel_ms": kms,
                        "nodes_per_s": len(pts) / wall,
                        "rms_err": float(np.sqrt(np.mean((est - fd[:, 2:4]) ** 2)))})
        else:
            row["note"] = "bias above 0.95e-3: RMS 1e-3 out of reach at this dt"
        res.append(row)
    return {"workload": "moving_bump_1521 (t = 0.1), identity data; bridge: Brownian-bridge exit test, "
                        "exits projected; exponential: exponential step lengths of mean dt with the bridge test; "
                        "pilot 1e5 paths", "runs": res}


def measure_steady():
    """The elliptic (steady) variant (eq. (2)): one-shot steady meshes, with
    the global steady solve (one sub-domain, the same banded LU) beside them
    -- the static bump on 2 x 2 sub-domains of a 64-cell grid (125 interface
    nodes, 2^18 paths) and the paper's ring at t = 0 on its 41 x 41 grid
    (2 x 2 sub-domains, 10^5 paths, equidistributed edges); dt 1e-4 with the
    bridge exit test."""
    import torch
    from paper_1402_0266_amd.mesh_run import DATA_EQUIDISTRIBUTED, DATA_IDENTITY, paper_ring_density, steady_mesh
    import paper_1402_0266_amd as fk
    res = {}
    for name, dens, px, m, n_paths, dt, horizon, bdry in (
            ("static_bump_125", W.static_bump(), 2, 32, 1 << 18, 1e-4, 3.0, DATA_IDENTITY),
            ("paper_ring_77", paper_ring_density(0.0), 2, 20, 100000, 1e-4, 20.0, DATA_EQUIDISTRIBUTED)):
        print(f"[bench] steady mesh: {name}", file=sys.stderr, flush=True)
        steady_mesh(dens, px, m, 256, dt, horizon, bdry=bdry)        # first-launch costs
        fk.fk_timing_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = steady_mesh(dens, px, m, n_paths, dt, horizon, bdry=bdry)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kms, _ = fk.fk_timing_last()
        fk.fk_timing_enable(False)
        q = fk.fk_mesh_quality(g["xi"], g["eta"]).cpu().numpy()
        # the global steady solve on the same grid: one sub-domain, no interfaces
        N = px * m
        empty = torch.empty(0, dtype=torch.float64, device="cuda")
        gx, gy = fk.subdomain_solve(dens, 0.0, float("inf"), 1, N, None, None, empty, empty, bdry_kind=bdry)
        qg = fk.fk_mesh_quality(gx, gy).cpu().numpy()
        se = torch.stack([g["se_xi"], g["se_eta"]]).cpu().numpy()
        res[name] = {"nodes": int(g["iface_xi"].numel()), "paths": n_paths, "dt": dt, "horizon": horizon,
                     "s": wall, "path_kernel_ms": kms, "survivors": int(g["survivors"]),
                     "min_jac": float(q[0]), "max_skew": float(q[1]), "se_median": float(np.median(se)),
                     "global_steady_min_jac": float(qg[0]), "global_steady_max_skew": float(qg[1]),
                     "max_diff_vs_global": float(max((g["xi"] - gx).abs().max(), (g["eta"] - gy).abs().max()))}
    return res


def measure_mesh_run():
    """The time-dependent mesh run, with the network and plain."""
    import torch
    from paper_1402_0266_amd.mesh_run import MeshRun, MeshRunConfig
    res = {}
    for name, kw in (("cv", {}), ("grid_cv", {"cv_form": "grid", "cv_stride": 2}),
                     ("grid_cv_keys", {"cv_form": "grid", "cv_stride": 2, "key_points": True, "key_gap": 8}),
                     ("plain", {"refit_every": 0})):
        cfg = MeshRunConfig(**kw)
        print(f"[bench] mesh run ({name}): {cfg.n_steps} steps", file=sys.stderr, flush=True)
        run = MeshRun(cfg, init_params=W.mlp_init(0) if cfg.refit_every else None)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for n in range(cfg.n_steps):
            run.step()
            if n % 50 == 49:
                print(f"[bench] mesh run ({name}): step {n + 1}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        q = run.qualities()
        _, se = run.interface_values()
        run.close()
        res[name] = {"s_total": wall, "ms_per_step": wall / cfg.n_steps * 1e3,
                     "min_jac_min": float(q[:, 0].min()), "min_jac_final": float(q[-1, 0]),
                     "max_skew_max": float(q[:, 1].max()), "max_skew_final": float(q[-1, 1]),
                     "min_jac_every_20": q[19::20, 0].round(4).tolist(),
                     "se_median": float(np.nanmedian(se)), "se_max": float(np.nanmax(se)),
                     "simulated_nodes_mean": float(np.mean(run.n_keys)) if run.n_keys else float(run.n_nodes)}
    res["config"] = ("8x8 sub-domains, 768-cell grid, 10689 interface nodes, two counter-rotating bumps A=30 "
                     "s2=0.003 frozen per step, 200 steps of 5e-4, 20 EM steps each, 2^14 paths/node; cv: "
                     "martingale form, stride 20, refit every 20 steps on mesh labels near the interfaces; grid_cv: "
                     "martingale form with the mesh's own gradient every 2 steps (no network); grid_cv_keys: the "
                     "same at the key points only (knots at most 8 nodes apart), the other interface nodes "
                     "interpolated")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cv", action="store_true", help="skip the control-variate measurement")
    ap.add_argument("--no-mesh-run", action="store_true", help="skip the time-dependent mesh run")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched 64-level launch")
    ap.add_argument("--no-paper-run", action="store_true", help="skip the paper's ring run")
    ap.add_argument("--no-bridge", action="store_true", help="skip the Brownian-bridge exit-test leg")
    ap.add_argument("--no-steady", action="store_true", help="skip the elliptic (steady) meshes")
    ap.add_argument("--paths", type=int, default=0, help="fix paths/node and skip the N* pilot (profiling)")
    ap.add_argument("--cv-kernels-only", action="store_true",
                    help="run only the control-variate kernels at the timed solve's size (profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (scales HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import torch
    import paper_1402_0266_amd as fk

    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n}))
        return

    if args.cv_kernels_only:
        print(json.dumps(cv_kernels_only(fk)))
        return

    wl = W.MOVING_BUMP_1521
    pts = wl.nodes()
    n_nodes = len(pts)
    fd = load_fd_reference(wl.name)
    dev = torch.device("cuda")
    ws = torch.empty(fk.fk_interface_workspace_bytes(n_nodes, wl.n_paths), dtype=torch.uint8, device=dev)

    dpts = torch.tensor(pts, dtype=torch.float64, device=dev)     # node coordinates stay resident

    def solve(n_paths):
        return fk.fk_interface_solve(wl.density, wl.data, dpts, wl.t, wl.dt, n_paths, wl.seed, workspace=ws)

    # ---- pilot at the configured paths/node: variance, bias, N* ----------------
    n_star = args.paths or wl.n_paths
    pilot = {"paths": wl.n_paths, "skipped": bool(args.paths)}
    if not args.paths:
        print(f"[bench] pilot: {n_nodes} nodes x {wl.n_paths} paths", file=sys.stderr, flush=True)
        r = solve(wl.n_paths)
        torch.cuda.synchronize()
        xi, eta = r["xi"].cpu().numpy(), r["eta"].cpu().numpy()
        se = np.stack([r["se_xi"].cpu().numpy(), r["se_eta"].cpu().numpy()], 1)
        var_mean = float(np.mean(se ** 2) * wl.n_paths)
        pilot["mean_score_var"] = var_mean
    if fd is not None and not args.paths:
        rms0 = rms_against(fd, xi, eta)
        b2 = max(0.0, rms0 ** 2 - var_mean / wl.n_paths)
        pilot.update({"rms": rms0, "bias": math.sqrt(b2), "fd_err_est": float(fd[:, 4:6].max())})
        if b2 >= 1e-6:
            n_star = wl.n_paths
            pilot["note"] = "bias floor reached: rate quoted at the configured paths"
        else:
            n_star = int(math.ceil(var_mean / (1e-6 - b2)))
    n_star = max(2, n_star)
    if n_star > wl.n_paths:
        ws = torch.empty(fk.fk_interface_workspace_bytes(n_nodes, n_star), dtype=torch.uint8, device=dev)

    # ---- warmup + timed steps at N* -------------------------------------------
    print(f"[bench] N* = {n_star}; warmup {args.warmup}, steps {args.steps}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        solve(n_star)
    torch.cuda.synchronize()
    fk.fk_timing_enable(True)
    kern_ms, red_ms, steps_total = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = solve(n_star)
        a, b = fk.fk_timing_last()
        kern_ms.append(a)
        red_ms.append(b)
        steps_total.append(int(r["total_steps"].item()))
        print(f"[bench] step: path kernel {a:.1f} ms, finalize {b:.2f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fk.fk_timing_enable(False)
    ms_per_step = wall / args.steps * 1e3
    value = n_nodes * args.steps / wall
    xi, eta = r["xi"].cpu().numpy(), r["eta"].cpu().numpy()
    rms = rms_against(fd, xi, eta) if fd is not None else None

    kms = float(np.mean(kern_ms))
    path_steps = float(np.mean(steps_total))
    achieved = FLOP_PER_STEP * path_steps / (kms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "moving_bump_1521: 4x4 sub-domains, 1521 interface nodes, moving bump A=20 s2=0.005, "
                        "t=0.1, dt=1e-5, plain MC, FP32 paths / FP64 estimator",
            "n_nodes": n_nodes, "paths_per_node": n_star, "rms_err": rms, "pilot": pilot,
            "path_steps_per_launch": path_steps,
            "path_steps_per_s": path_steps / (kms * 1e-3),
            "path_kernel_ms": kms, "finalize_kernel_ms": float(np.mean(red_ms)),
        },
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            # the same against the non-packed FP32 rate (one FMA per lane per cycle)
            "frac_of_unpacked_fp32": achieved / (FP32_PEAK_TFLOPS / 2),
            "traffic": (TRAFFIC_BYTES_PER_PATH * n_nodes * n_star
                        if kernel_source_hash() == TRAFFIC_SOURCE_HASH else None),
            "flop_per_path_step": FLOP_PER_STEP,
        },
    }
    if not args.no_cv and fd is not None:
        # the network as the deviation from the identity map (u_hat = (x, y) +
        # MLP); the plain-output network beside it
        out["cv"] = measure_cv(fk, wl, pts, fd, args.steps, args.warmup, identity_base=True)
        out["cv"]["identity_base"] = True
        pn = measure_cv(fk, wl, pts, fd, args.steps, args.warmup, identity_base=False)
        out["cv"]["plain_output_network"] = {k: pn[k] for k in ("form", "stride", "grad", "paths_per_node", "rms_err",
                                                                "nodes_per_s")}
        out["cv"]["plain_output_network"]["pilots"] = [
            {k: p.get(k) for k in ("form", "stride", "grad", "var_ratio", "n_star", "s_at_n_star")}
            for p in pn["pilots"]]
        # the fit the learned-control configuration names: 2000 Adam steps at lr 1e-3
        cf = measure_cv(fk, wl, pts, fd, args.steps, args.warmup, identity_base=True, schedule=((2000, 1e-3),))
        out["cv"]["fit_2000_steps"] = {k: cf[k] for k in ("form", "stride", "grad", "paths_per_node", "rms_err",
                                                          "nodes_per_s", "training")}
        out["cv"]["fit_2000_steps"]["pilots"] = [
            {k: p.get(k) for k in ("form", "stride", "grad", "var_ratio", "n_star", "s_at_n_star")}
            for p in cf["pilots"]]
    if not args.no_bridge and fd is not None:
        out["bridge"] = measure_bridge(fk, wl, pts, fd)
    if not args.no_mesh_run:
        out["mesh_run"] = measure_mesh_run()
    if not args.no_batched:
        out["batched"] = measure_batched(fk)
    if not args.no_paper_run:
        out["paper_run"] = measure_paper_run()
    if not args.no_steady:
        out["steady"] = measure_steady()
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, n_star)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
