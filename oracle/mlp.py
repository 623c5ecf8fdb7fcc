"""FP64 reference of the tile cost model (TEST INFRASTRUCTURE ONLY).

The paper has no cost model; this is the library's own component, written
here in plain numpy from the textbook definitions so the GPU kernels can be
checked against it:
  * a 68 -> 64 -> 64 -> 1 perceptron with ReLU hidden layers on standardised
    inputs x' = (x - mu) * inv_sd (mu, inv_sd fixed, not trained);
  * mean squared error over a minibatch, gradients by the chain rule
    (backpropagation), ReLU'(0) = 0;
  * Adam (Kingma & Ba, 2015, Algorithm 1): beta1 = 0.9, beta2 = 0.999,
    eps = 1e-8, bias-corrected moments, step t >= 1.
The flat parameter layout is the library's: mu[68], inv_sd[68], W1[64][68],
b1[64], W2[64][64], b2[64], w3[64], b3.
"""
from __future__ import annotations

import numpy as np

NF, NH = 68, 64
NORM = 2 * NF
SIZES = [("mu", (NF,)), ("inv_sd", (NF,)), ("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)),
         ("b2", (NH,)), ("w3", (NH,)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)  # 8777


def unpack(p: np.ndarray) -> dict:
    p = np.asarray(p, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[o:o + k].reshape(shape)
        o += k
    return out


def pack(d: dict) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def init_params(rng: np.random.Generator, mu=None, sd=None) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)), zero biases."""
    d = {"mu": np.zeros(NF) if mu is None else np.asarray(mu, dtype=np.float64),
         "inv_sd": np.ones(NF) if sd is None else 1.0 / np.asarray(sd, dtype=np.float64)}
    d["W1"] = rng.uniform(-1, 1, (NH, NF)) * np.sqrt(6.0 / NF)
    d["b1"] = np.zeros(NH)
    d["W2"] = rng.uniform(-1, 1, (NH, NH)) * np.sqrt(6.0 / NH)
    d["b2"] = np.zeros(NH)
    d["w3"] = rng.uniform(-1, 1, NH) * np.sqrt(6.0 / NH)
    d["b3"] = np.zeros(1)
    return pack(d)


def forward(p: np.ndarray, x: np.ndarray, keep: bool = False):
    """Predictions for rows of x; with keep=True also the pre-activations."""
    d = unpack(p)
    xs = (np.asarray(x, dtype=np.float64) - d["mu"]) * d["inv_sd"]
    a1 = xs @ d["W1"].T + d["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ d["W2"].T + d["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ d["w3"] + d["b3"][0]
    if keep:
        return y, (xs, a1, h1, a2, h2)
    return y


def loss_and_grad(p: np.ndarray, x: np.ndarray, t: np.ndarray):
    """Mean squared error and its gradient with respect to every parameter
    (zero for the standardisation entries)."""
    d = unpack(p)
    y, (xs, a1, h1, a2, h2) = forward(p, x, keep=True)
    B = len(y)
    e = y - np.asarray(t, dtype=np.float64)
    L = float(np.mean(e * e))
    gy = 2.0 * e / B
    g = {"mu": np.zeros(NF), "inv_sd": np.zeros(NF)}
    g["w3"] = h2.T @ gy
    g["b3"] = np.array([gy.sum()])
    ga2 = np.outer(gy, d["w3"]) * (a2 > 0)
    g["W2"] = ga2.T @ h1
    g["b2"] = ga2.sum(axis=0)
    ga1 = (ga2 @ d["W2"]) * (a1 > 0)
    g["W1"] = ga1.T @ xs
    g["b1"] = ga1.sum(axis=0)
    return L, pack(g)


def adam_step(p, m, v, g, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update of the trainable entries (index >= NORM)."""
    p, m, v = (np.array(a, dtype=np.float64) for a in (p, m, v))
    s = slice(NORM, None)
    m[s] = b1 * m[s] + (1 - b1) * g[s]
    v[s] = b2 * v[s] + (1 - b2) * g[s] * g[s]
    mh = m[s] / (1 - b1 ** t)
    vh = v[s] / (1 - b2 ** t)
    p[s] = p[s] - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def train_step(p, m, v, t: int, x, target, idx, lr: float):
    """The GPU step's definition: loss and Adam update on rows idx of (x, target)."""
    L, g = loss_and_grad(p, np.asarray(x)[idx], np.asarray(target)[idx])
    p, m, v = adam_step(p, m, v, g, t, lr)
    return L, p, m, v
