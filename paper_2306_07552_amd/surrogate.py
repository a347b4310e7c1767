"""Training of the collision surrogate on motions labelled by the simulator.

Every sample is one environment's next move: the features of (state, action)
from ``gal_features`` and, as the label, whether the exact column-grid test
of that move's candidate pose found a static contact (any bit of the step's
static contact mask).  The simulator itself generates the motions (random
actions, physics-only steps); the device MLP trains with its own MFMA
forward/backward kernels and Adam.  Calibration picks the skip threshold so
that no held-out positive would be skipped, with a safety factor.
"""
from __future__ import annotations

import math
import time
from typing import Dict, Tuple

import numpy as np


def generate(batch, num_samples: int, act_lim, seed: int = 0, device="cuda"):
    """(X int16 [n][2080] BF16 bits, y float32 [n]) from random-action rollouts."""
    import torch
    N = batch.num_envs
    steps = (num_samples + N - 1) // N
    X = torch.empty((steps * N, 2080), dtype=torch.int16, device=device)
    y = torch.empty(steps * N, dtype=torch.float32, device=device)
    out = {k: v for k, v in batch.alloc_outputs().items() if k not in ("depth", "rgb")}
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    lim = torch.tensor([act_lim[0], act_lim[1]] + [act_lim[2]] * 7, dtype=torch.float32,
                       device=device)
    act = torch.empty((N, 9), dtype=torch.float32, device=device)
    for k in range(steps):
        act.copy_((torch.rand((N, 9), generator=g, device=device) * 2 - 1) * lim)
        batch.features(act, X[k * N:(k + 1) * N])
        batch.step(act, out)
        y[k * N:(k + 1) * N] = (out["contact_static"] != 0).any(dim=1).float()
    return X[:num_samples], y[:num_samples]


def train(mlp, X, y, epochs: int = 2, batch_size: int = 4096, lr: float = 1e-3,
          pos_weight: float = 4.0, seed: int = 0, log=None) -> Dict[str, list]:
    import torch
    n = X.shape[0]
    g = torch.Generator(device=X.device)
    g.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=X.device)
    hist = []
    t0 = time.perf_counter()
    steps = 0
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g, device=X.device)
        acc = torch.zeros((), device=X.device)
        nb = 0
        for i in range(0, n - batch_size + 1, batch_size):
            idx = perm[i:i + batch_size]
            xb, yb = X[idx], y[idx]
            mlp.train_step(xb, yb, pos_weight, lr * 0.5 * (1 + math.cos(math.pi * (steps / max(1, epochs * (n // batch_size))))), loss)
            acc += loss[0]
            nb += 1
            steps += 1
        torch.cuda.synchronize()
        hist.append(float(acc) / max(nb, 1))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f} ({time.perf_counter() - t0:.1f} s)")
    return {"loss": hist, "seconds": time.perf_counter() - t0, "steps": steps}


def probabilities(mlp, X, chunk: int) -> "object":
    import torch
    z = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    for i in range(0, X.shape[0], chunk):
        xb = X[i:i + chunk]
        mlp.forward(xb, z[i:i + chunk], rows=xb.shape[0])
    return torch.sigmoid(z)


def calibrate(mlp, X, y, chunk: int, safety: float = 0.5, margin: float = 0.1) -> Tuple[float, dict]:
    """skip_below = min(tau - margin, safety * min positive probability), with
    tau the smallest probability of a held-out positive (no held-out positive
    may fall in the skip region)."""
    p = probabilities(mlp, X, chunk)
    pos = p[y > 0.5]
    neg = p[y <= 0.5]
    tau = float(pos.min()) if pos.numel() else 1.0
    skip_below = max(0.0, min(tau - margin, safety * tau))
    frac = float((neg <= skip_below).float().mean()) if neg.numel() else 0.0
    return skip_below, {"tau": tau, "skip_below": skip_below, "positives": int(pos.numel()),
                        "negatives": int(neg.numel()), "neg_skip_fraction": frac}
