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

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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

# HBM traffic of the path kernel from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
# (scaled by a plain 1 GiB copy: fetch x2.0, write x1.0), per path, valid only
# for the kernel sources it was measured on (hash below); otherwise null.
TRAFFIC_BYTES_PER_PATH = (0.4625 * 2**20 + 1071540.40625 * 1024) / (1521 * 73858)
TRAFFIC_SOURCE_HASH = "2253d4a70496d3d2"
KERNEL_SOURCES = ["paper_1402_0266_amd/csrc/fk_paths.hip", "paper_1402_0266_amd/csrc/fk_device.hpp",
                  "paper_1402_0266_amd/csrc/fk_internal.hpp"]


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


def cpu_baseline(wl, n_star, sample_nodes=96, sample_paths=2048):
    """The CPU oracle on a bounded sample: sample_nodes nodes spread evenly over the
    canonical order, sample_paths paths each,
    scaled to nodes/s at N* paths per node."""
    import oracle
    oracle.build()
    threads = min(16, os.cpu_count() or 1)
    pts = wl.nodes()
    sel = np.arange(0, len(pts), max(1, len(pts) // sample_nodes))[:sample_nodes]
    t0 = time.perf_counter()
    oracle.fk_solve(wl.density, wl.data, pts[sel], wl.t, wl.dt, sample_paths, wl.seed, node_ids=sel,
                    threads=threads)
    el = time.perf_counter() - t0
    nodes_per_s = len(sel) / el * (sample_paths / n_star)
    return {"value": nodes_per_s, "unit": "nodes/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(sel)} nodes (every {len(pts) // sample_nodes}th) x {sample_paths} paths, "
                      f"{el:.2f}s, scaled by {sample_paths}/{n_star} paths"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--paths", type=int, default=0, help="fix paths/node and skip the N* pilot (profiling)")
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

    wl = W.MOVING_BUMP_1521
    pts = wl.nodes()
    n_nodes = len(pts)
    fd = load_fd_reference(wl.name)
    dev = torch.device("cuda")
    ws = torch.empty(fk.fk_interface_workspace_bytes(n_nodes, wl.n_paths), dtype=torch.uint8, device=dev)

    def solve(n_paths):
        return fk.fk_interface_solve(wl.density, wl.data, pts, wl.t, wl.dt, n_paths, wl.seed, workspace=ws)

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
        print(f"[bench] step: path kernel {a:.1f} ms, reduce {b:.2f} ms", file=sys.stderr, flush=True)
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
            "path_kernel_ms": kms, "reduce_kernel_ms": float(np.mean(red_ms)),
        },
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": (TRAFFIC_BYTES_PER_PATH * n_nodes * n_star
                        if kernel_source_hash() == TRAFFIC_SOURCE_HASH else None),
            "flop_per_path_step": FLOP_PER_STEP,
        },
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, n_star)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
