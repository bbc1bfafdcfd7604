"""Control-variate pipeline on the GPU: training labels from batched plain
Monte-Carlo interface solves, network training, and the control-variate
solve.  Every step runs in libfk.so kernels; this module only sequences the
calls.
"""
from __future__ import annotations

import numpy as np

from . import FkBatch, FkCv, fk_interface_solve_cv  # noqa: F401

LABEL_LEVEL_BASE = 1 << 20   # Philox level tags of label paths, disjoint from solve levels


def make_labels(density, data, nodes, t_levels, dt, n_paths, seed=0, device="cuda"):
    """Plain-MC estimates at every node for every time level, as training
    data: returns device FP32 tensors txy [n, 3] (t, x, y) and target [n, 2]
    (xi, eta), levels concatenated in order."""
    import torch
    levels = [(density, float(t), 0.0, nodes, LABEL_LEVEL_BASE + m) for m, t in enumerate(t_levels)]
    batch = FkBatch(levels, data, dt, n_paths, seed=seed, device=device)
    out = batch.run()
    n = len(nodes)
    t_col = np.repeat(np.asarray(t_levels, dtype=np.float64), n)
    xy = np.tile(np.asarray(nodes, dtype=np.float64), (len(t_levels), 1))
    txy = torch.tensor(np.concatenate([t_col[:, None], xy], 1), dtype=torch.float32, device=device)
    target = torch.stack([out["xi"], out["eta"]], 1).to(torch.float32)
    batch.close()
    return txy, target


def train(cv: FkCv, txy, target, steps=2000, batch=8192, lr=1e-3, seed=0):
    """Adam on minibatches; returns the per-step minibatch losses (device)."""
    return cv.train(txy, target, steps=steps, batch=batch, lr=lr, seed=seed)


# The default fit: Adam stages of (steps, learning rate), a constant rate and
# two decays; the moments and the step count carry over from stage to stage.
TRAIN_SCHEDULE = ((8000, 2e-3), (4000, 5e-4), (4000, 1e-4))


def train_schedule(cv: FkCv, txy, target, schedule=TRAIN_SCHEDULE, batch=8192, seed=0):
    """Adam through the stages of ``schedule``; returns the per-step
    minibatch losses of all stages (device), in order."""
    import torch
    losses = [cv.train(txy, target, steps=n, batch=batch, lr=lr, seed=seed + i) for i, (n, lr) in enumerate(schedule)]
    return torch.cat(losses)
