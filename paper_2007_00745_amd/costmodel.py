"""Tile cost model: data collection, training and evaluation.

Host-side orchestration only.  Rendering with per-tile cost logs, probe
features, log-cost targets, input standardisation, every training step (the
forward pass, backpropagation and the Adam update) and inference run in the
library's HIP kernels; this module draws the random numbers (initial weights,
minibatch order) and loops over epochs.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import native

NF, NH = native.NFEAT, 64


def init_params(seed: int) -> torch.Tensor:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases; the
    standardisation entries are set later from the data."""
    rng = np.random.default_rng(seed)
    p = np.zeros(native.MLP_PARAMS, dtype=np.float32)
    p[NF:2 * NF] = 1.0
    o = native.MLP_NORM
    p[o:o + NH * NF] = rng.uniform(-1, 1, NH * NF) * math.sqrt(6.0 / NF)
    o += NH * NF + NH
    p[o:o + NH * NH] = rng.uniform(-1, 1, NH * NH) * math.sqrt(6.0 / NH)
    o += NH * NH + NH
    p[o:o + NH] = rng.uniform(-1, 1, NH) * math.sqrt(6.0 / NH)
    return torch.tensor(p, device="cuda")


def collect(views, tuning: dict | None = None, probe_cap: int = 0):
    """Render the views once with per-tile cost logging; return (features,
    ln-cost targets, raw costs, plan)."""
    plan = native.Plan(views, tuning)
    out = torch.empty(max(plan.out_size(), 1), dtype=torch.int32, device="cuda")
    cost = torch.empty(max(plan.ntiles, 1), dtype=torch.int64, device="cuda")
    plan.launch(out, tile_cost=cost)
    feat = plan.features(probe_cap=probe_cap)
    target = native.cost_targets(cost[:plan.ntiles])
    del out
    return feat, target, cost[:plan.ntiles], plan


def train(feat, target, epochs: int = 30, batch: int = 512, lr: float = 1e-3, seed: int = 0,
          max_samples: int = 200_000, params=None, log=None):
    """Minibatch Adam on the mean squared error of predicted ln(cost).
    Returns (params, per-epoch mean losses)."""
    rng = np.random.default_rng(seed)
    N = int(feat.shape[0])
    sel = rng.choice(N, min(N, max_samples), replace=False)
    if params is None:
        params = init_params(seed)
        native.mlp_set_norm(params, feat)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    work = torch.empty(native.mlp_work_floats(batch), dtype=torch.float32, device="cuda")
    steps_per_epoch = len(sel) // batch
    losses = torch.zeros(max(1, epochs * steps_per_epoch), dtype=torch.float32, device="cuda")
    t = 0
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(sel).astype(np.int32), device="cuda")
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            native.mlp_train_step(params, m, v, t + 1, feat, target, idx, lr,
                                  loss=losses[t:t + 1], work=work)
            t += 1
        if log is not None:
            log(f"epoch {ep}: loss {losses[t - steps_per_epoch:t].mean().item():.4f}")
    per_epoch = losses[:t].view(epochs, steps_per_epoch).mean(dim=1).cpu().tolist() if t else []
    return params, per_epoch


def spearman(a, b) -> float:
    ra = np.argsort(np.argsort(a, kind="stable"), kind="stable").astype(np.float64)
    rb = np.argsort(np.argsort(b, kind="stable"), kind="stable").astype(np.float64)
    ra -= ra.mean()
    rb -= rb.mean()
    return float((ra * rb).sum() / math.sqrt((ra * ra).sum() * (rb * rb).sum()))


def evaluate(params, feat, target) -> dict:
    pred = native.mlp_forward(params, feat).cpu().numpy().astype(np.float64)
    tgt = target.cpu().numpy().astype(np.float64)
    return {"rmse_ln_cost": float(np.sqrt(np.mean((pred - tgt) ** 2))),
            "spearman": spearman(pred, tgt), "tiles": int(len(tgt))}
