"""Training of the collision surrogate on motions labelled by the simulator.

Every sample is one environment's next move: the features of (state, action)
from ``gal_features`` and, as the label, whether the column-grid test of that
move's candidate pose found a static contact (any bit of the step's static
contact mask).  The simulator itself generates the motions (random actions,
physics-only steps) and labels them; the device MLP trains with its own MFMA
forward/backward kernels and Adam.

Training labels carry a safety margin: they come from a labelling batch of
the same scenes whose sphere classes are the real radii plus ``label_margin``
(every sphere inflated), with the real largest radius appended as its last
class so that its occupancy lattice, and hence every feature, is the one a
plain batch computes.  The network thus learns a band around every obstacle
as "contact", and true contacts sit inside that band rather than on its edge.
Calibration uses true labels: the skip threshold lies below the smallest
held-out true-positive probability, by a safety factor and by the spread of
the observed lower tail of the positives (``skip_threshold``).
"""
from __future__ import annotations

import math
import time
from typing import Dict, Tuple

import numpy as np


def generate(batch, num_samples: int, act_lim, seed: int = 0, device="cuda"):
    """(X int16 [n][2112] BF16 bits, y float32 [n]) from random-action rollouts."""
    import torch
    N = batch.num_envs
    steps = (num_samples + N - 1) // N
    X = torch.empty((steps * N, 2112), dtype=torch.int16, device=device)
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


def skip_threshold(pos_p, safety: float = 0.25, tail_quantile: float = 0.001) -> Tuple[float, float]:
    """Skip threshold from the probabilities of true held-out contacts.

    tau is the smallest of them.  The threshold is the lower of safety * tau
    and the probability whose logit lies below tau's by the spread of the
    observed tail (the logit distance from tau up to the positives'
    ``tail_quantile`` quantile): the tail seen between that quantile and the
    minimum is assumed to continue at least as far again below it, which is
    where unseen contacts of a larger deployment fall.  Returns
    (skip_below, tau)."""
    import torch
    pos = torch.as_tensor(pos_p).double().flatten()
    if pos.numel() == 0:
        return safety, 1.0
    tau = float(pos.min())
    q = float(torch.quantile(pos, tail_quantile))
    eps = 1e-30
    logit = lambda v: math.log(max(v, eps)) - math.log(max(1.0 - v, eps))
    z = logit(tau) - max(logit(q) - logit(tau), 0.0)
    ext = 1.0 / (1.0 + math.exp(-z))
    return min(safety * tau, ext), tau


def calibrate(mlp, X, y, chunk: int, safety: float = 0.25, margin: float = 0.1) -> Tuple[float, dict]:
    """Skip threshold from true-labelled held-out data (``skip_threshold``):
    the exact check is skipped for p <= skip_below, so no held-out positive
    is skipped and the unseen tail keeps room below the smallest one.
    Predicted contacts (p >= skip_below + margin) and the band between the
    two, the margin, both run the exact check, so only skip_below routes
    work."""
    import torch
    p = probabilities(mlp, X, chunk)
    pos = p[y > 0.5]
    neg = p[y <= 0.5]
    skip_below, tau = skip_threshold(pos, safety)
    frac = float((neg <= skip_below).float().mean()) if neg.numel() else 0.0
    q = torch.tensor([0.0, 0.001, 0.01, 0.1], device=p.device)
    pq = [round(float(v), 6) for v in torch.quantile(pos.double(), q.double())] if pos.numel() else []
    return skip_below, {"tau": tau, "skip_below": skip_below, "decide_contact_above": skip_below + margin,
                        "positives": int(pos.numel()), "negatives": int(neg.numel()),
                        "neg_skip_fraction": frac, "pos_quantiles_0_0.1_1_10pct": pq}


def labelling_consts(consts: dict, label_margin: float) -> dict:
    """Batch constants whose sphere classes are inflated by ``label_margin``,
    with the real largest radius as the last class (the lattice class)."""
    rc = [float(r) for r in consts["radius_classes"]]
    out = dict(consts)
    out["radius_classes"] = tuple([r + label_margin for r in rc] + [rc[-1]])
    return out


def fit(robot, consts, cfg, train_envs, holdout_envs, samples: int = 1 << 24, epochs: int = 4,
        holdout_samples: int = 1 << 22, pos_weight: float = 8.0, lr: float = 1e-3,
        label_margin: float = 0.12, max_rows: int = 4096, seed: int = 5, log=None):
    """The surrogate recipe: rollouts of ``train_envs`` labelled with the
    safety margin, weighted logistic loss with Adam (cosine schedule), then
    the conservative calibration on true-labelled rollouts of
    ``holdout_envs`` (other scenes).  Returns (mlp, skip_below, info)."""
    import torch
    from . import gal, scenegen as sg
    t0 = time.perf_counter()
    tr = gal.Batch(robot, sg.make_scene_set(cfg, train_envs),
                   labelling_consts(consts, label_margin) if label_margin > 0 else consts)
    X, y = generate(tr, samples, cfg.act_lim, seed=seed + 2)
    pos_rate = float(y.mean())
    mlp = gal.Mlp(max_rows=max_rows, seed=seed)
    hist = train(mlp, X, y, epochs=epochs, batch_size=4096, lr=lr, pos_weight=pos_weight, log=log)
    del X, y, tr
    torch.cuda.empty_cache()
    ho = gal.Batch(robot, sg.make_scene_set(cfg, holdout_envs), consts)
    Xh, yh = generate(ho, holdout_samples, cfg.act_lim, seed=seed + 3)
    skip_below, info = calibrate(mlp, Xh, yh, chunk=4096)
    del Xh, yh, ho
    info.update(train_samples=samples, epochs=epochs, pos_weight=pos_weight, label_margin=label_margin,
                train_loss=[round(v, 5) for v in hist["loss"]],
                train_seconds=round(hist["seconds"], 2), positive_rate=round(pos_rate, 4),
                setup_seconds=round(time.perf_counter() - t0, 1))
    return mlp, skip_below, info
