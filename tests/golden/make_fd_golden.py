"""Writes the finite-difference reference values at the interface nodes.

Calls only the CPU oracle (oracle.fd_solve, ADI with central differences):
solves on n and 2n cells per side and stores the Richardson-extrapolated
values with the error estimate |u_2n - u_n| / 3.

    python tests/golden/make_fd_golden.py [workload ...]
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SETTINGS = {
    # workload: (coarse n, time step of the ADI solve)
    "static_bump_31": (256, 1e-5),
    "moving_bump_1521": (512, 1e-5),
}


def write(name: str) -> str:
    wl = {"static_bump_31": W.STATIC_BUMP_31, "moving_bump_1521": W.MOVING_BUMP_1521}[name]
    n, dtau = SETTINGS[name]
    pts = wl.nodes()
    t0 = time.time()
    val, err = oracle.fd_reference_at(wl.density, wl.data, wl.t, pts, n_coarse=n, dtau=dtau)
    path = os.path.join(HERE, f"{name}_fd.txt")
    with open(path, "w") as f:
        f.write(f"# FD reference (ADI, central differences, Richardson on n={n},{2 * n}; dtau={dtau})\n")
        f.write(f"# workload {name}: t={wl.t}; density kind {wl.density.kind} params {[float(v) for v in wl.density.params()]}\n")
        f.write("# written by tests/golden/make_fd_golden.py from the CPU oracle only\n")
        f.write("# x y xi eta err_xi err_eta\n")
        for p, v, e in zip(pts, val, err):
            f.write(f"{p[0]:.17g} {p[1]:.17g} {v[0]:.17g} {v[1]:.17g} {e[0]:.3e} {e[1]:.3e}\n")
    print(f"{name}: {len(pts)} nodes in {time.time() - t0:.1f}s; max error estimate {err.max():.2e}", flush=True)
    return path


def load(name: str, root: str = HERE) -> np.ndarray:
    """[n, 6] array: x, y, xi, eta, err_xi, err_eta."""
    return np.loadtxt(os.path.join(root, f"{name}_fd.txt"))


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(SETTINGS)):
        write(nm)
