"""Pins of the FP64 cost-model reference (oracle/mlp.py) to facts outside it:
central finite differences of the loss, closed-form gradients where the
network is degenerate, and Adam's first step, whose size is known exactly."""
import numpy as np
import pytest

from oracle import mlp


def _data(seed, n=24):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, mlp.NF))
    t = rng.normal(size=n)
    p = mlp.init_params(rng, mu=rng.normal(size=mlp.NF) * 0.1, sd=rng.uniform(0.5, 2, mlp.NF))
    return p, x, t


def test_layout():
    assert mlp.NPARAMS == 8777
    assert mlp.NPARAMS - mlp.NORM == 68 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 8641
    p = np.arange(mlp.NPARAMS, dtype=np.float64)
    assert np.array_equal(mlp.pack(mlp.unpack(p)), p)


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_central_differences(seed):
    p, x, t = _data(seed)
    L, g = mlp.loss_and_grad(p, x, t)
    rng = np.random.default_rng(100 + seed)
    # a sample of coordinates from every block of trainable parameters
    idx = np.concatenate([rng.choice(np.arange(lo, hi), 12, replace=False) for lo, hi in
                          ((136, 4488), (4488, 4552), (4552, 8648), (8648, 8712),
                           (8712, 8776))] + [np.array([8776])])
    eps = 1e-6
    for j in idx:
        pp, pm = p.copy(), p.copy()
        pp[j] += eps
        pm[j] -= eps
        fd = (mlp.loss_and_grad(pp, x, t)[0] - mlp.loss_and_grad(pm, x, t)[0]) / (2 * eps)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd)), (j, fd, g[j])
    assert np.all(g[:mlp.NORM] == 0)


def test_zero_weights_closed_form():
    # With all weights and biases zero except b3 = c, y = c for every row, so
    # dL/db3 = 2 mean(c - t) and every other gradient vanishes (ReLU'(0) = 0).
    rng = np.random.default_rng(3)
    x = rng.normal(size=(10, mlp.NF))
    t = rng.normal(size=10)
    d = mlp.unpack(np.zeros(mlp.NPARAMS))
    d["inv_sd"] = np.ones(mlp.NF)
    d["b3"] = np.array([0.7])
    p = mlp.pack(d)
    L, g = mlp.loss_and_grad(p, x, t)
    assert np.isclose(L, np.mean((0.7 - t) ** 2), rtol=0, atol=1e-15)
    assert np.isclose(g[-1], 2 * np.mean(0.7 - t), rtol=0, atol=1e-15)
    assert np.all(g[:-1] == 0)


def test_linear_regime_closed_form():
    # If every hidden pre-activation is positive, the network is affine in b3 and w3;
    # check dL/dw3 = h2^T (2 e / B) against an explicit double loop.
    p, x, t = _data(5)
    d = mlp.unpack(p)
    d["b1"] = np.full(64, 50.0)
    d["W2"] = np.abs(d["W2"])
    d["b2"] = np.full(64, 50.0)
    p = mlp.pack(d)
    y, (xs, a1, h1, a2, h2) = mlp.forward(p, x, keep=True)
    assert np.all(a1 > 0) and np.all(a2 > 0)
    L, g = mlp.loss_and_grad(p, x, t)
    e = y - t
    for o in range(0, 64, 9):
        want = sum(2 * e[b] / len(t) * h2[b, o] for b in range(len(t)))
        assert np.isclose(g[8712 + o], want, rtol=1e-12)


def test_adam_first_step_size():
    # At t = 1 the bias-corrected moments are g and g^2, so the step is exactly
    # lr * g / (|g| + eps): about lr against the sign of the gradient.
    p, x, t = _data(7)
    L, g = mlp.loss_and_grad(p, x, t)
    z = np.zeros_like(p)
    p1, m1, v1 = mlp.adam_step(p, z, z, g, 1, 1e-3)
    s = slice(mlp.NORM, None)
    assert np.allclose((p - p1)[s], 1e-3 * g[s] / (np.abs(g[s]) + 1e-8), rtol=1e-9, atol=0)
    big = np.abs(g[s]) > 1e-4
    assert np.allclose((p - p1)[s][big], 1e-3 * np.sign(g[s][big]), rtol=1e-3, atol=0)
    assert np.allclose(m1[s], 0.1 * g[s]) and np.allclose(v1[s], 0.001 * g[s] ** 2)
    assert np.array_equal(p1[:mlp.NORM], p[:mlp.NORM])


def test_training_reduces_loss():
    rng = np.random.default_rng(9)
    x = rng.normal(size=(256, mlp.NF))
    w = rng.normal(size=mlp.NF)
    t = np.tanh(x @ w / 8.0) * 3.0
    p = mlp.init_params(rng)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    L0 = mlp.loss_and_grad(p, x, t)[0]
    for step in range(1, 201):
        idx = rng.choice(256, 64, replace=False)
        _, p, m, v = mlp.train_step(p, m, v, step, x, t, idx, 3e-3)
    assert mlp.loss_and_grad(p, x, t)[0] < 0.2 * L0
