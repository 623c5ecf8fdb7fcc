"""Pins of the FP64 cost-model reference (oracle/mlp.py) to facts outside it:
a hand-computed forward pass and hand-computed gradients of a tiny network with
non-trivial standardisation and non-zero biases; central finite differences of
the loss; closed-form gradients where the network is degenerate; Adam's step,
whose size is known exactly at t = 1 and, for a constant gradient, at every t.
Planted mistakes in copies of oracle/mlp.py (dropped standardisation, a missing
bias, Adam's bias correction without the power of t, ...) must each fail a pin."""
import importlib.util
import os

import numpy as np
import pytest

from oracle import mlp

MLP_SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "oracle", "mlp.py")


def _data(M, seed, n=24):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, M.NF))
    t = rng.normal(size=n)
    p = M.init_params(rng, mu=rng.normal(size=M.NF) * 0.1, sd=rng.uniform(0.5, 2, M.NF))
    # non-zero biases, so that every bias term shows in the outputs and gradients
    d = M.unpack(p)
    d["b1"] = rng.normal(size=M.NH) * 0.3
    d["b2"] = rng.normal(size=M.NH) * 0.3
    d["b3"] = np.array([0.4])
    return M.pack(d), x, t


# ---- the tiny network ---------------------------------------------------------------
# Inputs 0..3 are standardised with mu = (1, 2, -1, 0.5) and inv_sd = (0.5, 2, 4, 0.25);
# hidden unit k < 4 of layer 1 reads standardised input k alone (weight 1), unit 4 is
# the constant relu(b1[4]) = 0.5, unit 5 = relu(x'[0] - 1) sits exactly at 0, every
# other unit is dead (b1 = -1).  Layer 2:
#   unit 0 = relu(h1[0] + h1[1] + h1[5] - 0.5),  unit 1 = relu(2 h1[4] - h1[0]),
#   unit 2 = relu(h1[1] + 2),  unit 3 = relu(h1[0] - 1.25) (exactly 0), the rest 0;
#   y = 2 h2[0] + 5 h2[1] - h2[2] + 3 h2[3] + 0.75.
# For x = (3, 1, -2, 5, 0, ...):
#   x' = (1, -2, -4, 1.125), a1 = (1.25, 1, -3, -0.875, 0.5, 0), h1 = (1.25, 1, 0, 0, 0.5, 0),
#   a2 = (1.75, -0.25, 3, 0), h2 = (1.75, 0, 3, 0), y = 3.5 - 3 + 0.75 = 1.25.
# Every value is a short binary fraction, so FP64 gives them exactly.

def _tiny(M):
    d = M.unpack(np.zeros(M.NPARAMS))
    d["mu"] = np.zeros(M.NF)
    d["inv_sd"] = np.ones(M.NF)
    d["mu"][:4] = [1.0, 2.0, -1.0, 0.5]
    d["inv_sd"][:4] = [0.5, 2.0, 4.0, 0.25]
    d["W1"] = np.zeros((M.NH, M.NF))
    for k in range(4):
        d["W1"][k, k] = 1.0
    d["W1"][5, 0] = 1.0              # a1[5] = x'[0] - 1 = 0 exactly: ReLU'(0) = 0 is used
    d["b1"] = np.full(M.NH, -1.0)
    d["b1"][:5] = [0.25, 3.0, 1.0, -2.0, 0.5]
    d["W2"] = np.zeros((M.NH, M.NH))
    d["W2"][0, 0] = d["W2"][0, 1] = 1.0
    d["W2"][1, 4], d["W2"][1, 0] = 2.0, -1.0
    d["W2"][2, 1] = 1.0
    d["W2"][0, 5] = 1.0              # from the unit at a1 = 0
    d["W2"][3, 0] = 1.0              # a2[3] = h1[0] - 1.25 = 0 exactly
    d["b2"] = np.zeros(M.NH)
    d["b2"][:4] = [-0.5, 0.0, 2.0, -1.25]
    d["w3"] = np.zeros(M.NH)
    d["w3"][:4] = [2.0, 5.0, -1.0, 3.0]
    d["b3"] = np.array([0.75])
    x = np.zeros((1, M.NF))
    x[0, :4] = [3.0, 1.0, -2.0, 5.0]
    return M.pack(d), x


def pin_tiny_forward(M):
    p, x = _tiny(M)
    y, (xs, a1, h1, a2, h2) = M.forward(p, x, keep=True)
    assert np.array_equal(xs[0, :4], [1.0, -2.0, -4.0, 1.125])
    assert np.array_equal(a1[0, :6], [1.25, 1.0, -3.0, -0.875, 0.5, 0.0])
    assert np.array_equal(h1[0, :5], [1.25, 1.0, 0.0, 0.0, 0.5]) and not h1[0, 5:].any()
    assert np.array_equal(a2[0, :4], [1.75, -0.25, 3.0, 0.0]) and not h2[0, 3:].any()
    assert y[0] == 1.25


def pin_tiny_gradients(M):
    # L = (y - t)^2 with t = 0.25, so dL/dy = 2 (1.25 - 0.25) = 2.  Written out by the
    # chain rule on the tiny network: units 0 and 2 of layer 2 are active, unit 1 is not;
    # units 0, 1 and 4 of layer 1 are active.  Units at a pre-activation of exactly 0
    # (layer 1 unit 5, layer 2 unit 3) pass no gradient: ReLU'(0) = 0.
    p, x = _tiny(M)
    L, g = M.loss_and_grad(p, x, np.array([0.25]))
    G = M.unpack(g)
    assert L == 1.0
    assert G["b3"][0] == 2.0
    assert np.array_equal(G["w3"][:4], [2.0 * 1.75, 0.0, 2.0 * 3.0, 0.0])
    assert np.array_equal(G["b2"][:3], [2.0 * 2.0, 0.0, 2.0 * -1.0]) and not G["b2"][3:].any()
    # dL/da1[k] = sum_j dL/da2[j] W2[j, k] on active units: unit 0 gets 4 (via a2[0]);
    # unit 1 gets 4 - 2 = 2 (via a2[0] and a2[2]); unit 4 only feeds the inactive a2[1]
    assert np.array_equal(G["b1"][:5], [4.0, 2.0, 0.0, 0.0, 0.0]) and not G["b1"][5:].any()
    # dL/dW1[k, i] = dL/da1[k] * x'[i]: the standardised inputs, not the raw ones
    assert np.array_equal(G["W1"][0, :4], [4.0, -8.0, -16.0, 4.5])
    assert np.array_equal(G["W1"][1, :4], [2.0, -4.0, -8.0, 2.25])
    assert not G["W1"][2:].any()
    # dL/dW2[j, k] = dL/da2[j] * h1[k]
    assert np.array_equal(G["W2"][0, [0, 1, 4, 5]], [4.0 * 1.25, 4.0, 4.0 * 0.5, 0.0])
    assert np.array_equal(G["W2"][2, [0, 1, 4]], [-2.0 * 1.25, -2.0, -2.0 * 0.5])
    assert not G["W2"][1].any() and not G["W2"][3].any()
    assert not g[:M.NORM].any()


def pin_gradient_matches_central_differences(M, seed=1):
    p, x, t = _data(M, seed)
    L, g = M.loss_and_grad(p, x, t)
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
        fd = (M.loss_and_grad(pp, x, t)[0] - M.loss_and_grad(pm, x, t)[0]) / (2 * eps)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(fd)), (j, fd, g[j])
    assert np.all(g[:M.NORM] == 0)


def pin_zero_weights_closed_form(M):
    # With all weights and biases zero except b3 = c, y = c for every row, so
    # dL/db3 = 2 mean(c - t) and every other gradient vanishes (ReLU'(0) = 0).
    rng = np.random.default_rng(3)
    x = rng.normal(size=(10, M.NF))
    t = rng.normal(size=10)
    d = M.unpack(np.zeros(M.NPARAMS))
    d["inv_sd"] = np.ones(M.NF)
    d["b3"] = np.array([0.7])
    p = M.pack(d)
    L, g = M.loss_and_grad(p, x, t)
    assert np.isclose(L, np.mean((0.7 - t) ** 2), rtol=0, atol=1e-15)
    assert np.isclose(g[-1], 2 * np.mean(0.7 - t), rtol=0, atol=1e-15)
    assert np.all(g[:-1] == 0)


def pin_linear_regime_closed_form(M):
    # If every hidden pre-activation is positive, the network is affine in b3 and w3;
    # check dL/dw3 = h2^T (2 e / B) against an explicit double loop.
    p, x, t = _data(M, 5)
    d = M.unpack(p)
    d["b1"] = np.full(64, 50.0)
    d["W2"] = np.abs(d["W2"])
    d["b2"] = np.full(64, 50.0)
    p = M.pack(d)
    y, (xs, a1, h1, a2, h2) = M.forward(p, x, keep=True)
    assert np.all(a1 > 0) and np.all(a2 > 0)
    L, g = M.loss_and_grad(p, x, t)
    e = y - t
    for o in range(0, 64, 9):
        want = sum(2 * e[b] / len(t) * h2[b, o] for b in range(len(t)))
        assert np.isclose(g[8712 + o], want, rtol=1e-12)


def pin_adam_first_step_size(M):
    # At t = 1 the bias-corrected moments are g and g^2, so the step is exactly
    # lr * g / (|g| + eps): about lr against the sign of the gradient.
    p, x, t = _data(M, 7)
    L, g = M.loss_and_grad(p, x, t)
    z = np.zeros_like(p)
    p1, m1, v1 = M.adam_step(p, z, z, g, 1, 1e-3)
    s = slice(M.NORM, None)
    assert np.allclose((p - p1)[s], 1e-3 * g[s] / (np.abs(g[s]) + 1e-8), rtol=1e-9, atol=0)
    big = np.abs(g[s]) > 1e-4
    assert np.allclose((p - p1)[s][big], 1e-3 * np.sign(g[s][big]), rtol=1e-3, atol=0)
    assert np.allclose(m1[s], 0.1 * g[s]) and np.allclose(v1[s], 0.001 * g[s] ** 2)
    assert np.array_equal(p1[:M.NORM], p[:M.NORM])


def pin_adam_constant_gradient(M):
    # With the same gradient g at every step, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2,
    # so the bias-corrected moments are g and g^2 at every t and every step is
    # lr * g / (|g| + eps) (Kingma & Ba, Sec. 3: the correction removes the start-up bias).
    rng = np.random.default_rng(8)
    g = np.zeros(M.NPARAMS)
    g[M.NORM:] = rng.normal(size=M.NPARAMS - M.NORM) * 10.0 ** rng.uniform(-3, 1, M.NPARAMS - M.NORM)
    p = rng.normal(size=M.NPARAMS)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    s = slice(M.NORM, None)
    step = 2e-3 * g[s] / (np.abs(g[s]) + 1e-8)
    for t in range(1, 11):
        p1, m, v = M.adam_step(p, m, v, g, t, 2e-3)
        assert np.allclose((p - p1)[s], step, rtol=1e-9, atol=1e-15), f"t = {t}"
        p = p1


def pin_training_reduces_loss(M):
    rng = np.random.default_rng(9)
    x = rng.normal(size=(256, M.NF))
    w = rng.normal(size=M.NF)
    t = np.tanh(x @ w / 8.0) * 3.0
    p = M.init_params(rng)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    L0 = M.loss_and_grad(p, x, t)[0]
    for step in range(1, 201):
        idx = rng.choice(256, 64, replace=False)
        _, p, m, v = M.train_step(p, m, v, step, x, t, idx, 3e-3)
    assert M.loss_and_grad(p, x, t)[0] < 0.2 * L0


PINS = [pin_tiny_forward, pin_tiny_gradients, pin_gradient_matches_central_differences,
        pin_zero_weights_closed_form, pin_linear_regime_closed_form, pin_adam_first_step_size,
        pin_adam_constant_gradient, pin_training_reduces_loss]


def test_layout():
    assert mlp.NPARAMS == 8777
    assert mlp.NPARAMS - mlp.NORM == 68 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 8641
    p = np.arange(mlp.NPARAMS, dtype=np.float64)
    assert np.array_equal(mlp.pack(mlp.unpack(p)), p)


@pytest.mark.parametrize("pin", PINS, ids=[f.__name__ for f in PINS])
def test_pin(pin):
    pin(mlp)


def test_gradient_matches_central_differences_second_seed():
    pin_gradient_matches_central_differences(mlp, seed=2)


# ---- planted mistakes ---------------------------------------------------------------
MUTATIONS = {
    "no_standardisation": ('xs = (np.asarray(x, dtype=np.float64) - d["mu"]) * d["inv_sd"]',
                           'xs = np.asarray(x, dtype=np.float64)'),
    "divide_by_inv_sd": ('xs = (np.asarray(x, dtype=np.float64) - d["mu"]) * d["inv_sd"]',
                         'xs = (np.asarray(x, dtype=np.float64) - d["mu"]) / d["inv_sd"]'),
    "no_mean_shift": ('xs = (np.asarray(x, dtype=np.float64) - d["mu"]) * d["inv_sd"]',
                      'xs = np.asarray(x, dtype=np.float64) * d["inv_sd"]'),
    "missing_b1": ('a1 = xs @ d["W1"].T + d["b1"]', 'a1 = xs @ d["W1"].T'),
    "missing_b2": ('a2 = h1 @ d["W2"].T + d["b2"]', 'a2 = h1 @ d["W2"].T'),
    "missing_b3": ('y = h2 @ d["w3"] + d["b3"][0]', 'y = h2 @ d["w3"]'),
    "transposed_W2": ('a2 = h1 @ d["W2"].T + d["b2"]', 'a2 = h1 @ d["W2"] + d["b2"]'),
    "adam_m_without_power_of_t": ("mh = m[s] / (1 - b1 ** t)", "mh = m[s] / (1 - b1)"),
    "adam_v_without_power_of_t": ("vh = v[s] / (1 - b2 ** t)", "vh = v[s] / (1 - b2)"),
    "adam_no_bias_correction": ("mh = m[s] / (1 - b1 ** t)", "mh = m[s]"),
    "adam_eps_inside_sqrt": ("p[s] = p[s] - lr * mh / (np.sqrt(vh) + eps)",
                             "p[s] = p[s] - lr * mh / np.sqrt(vh + eps)"),
    "relu_grad_at_zero_is_one": ('ga1 = (ga2 @ d["W2"]) * (a1 > 0)',
                                 'ga1 = (ga2 @ d["W2"]) * (a1 >= 0)'),
    "relu2_grad_at_zero_is_one": ('ga2 = np.outer(gy, d["w3"]) * (a2 > 0)',
                                  'ga2 = np.outer(gy, d["w3"]) * (a2 >= 0)'),
    "W1_grad_on_raw_inputs": ('g["W1"] = ga1.T @ xs',
                              'g["W1"] = ga1.T @ np.asarray(x, dtype=np.float64)'),
    "loss_not_mean": ("gy = 2.0 * e / B", "gy = 2.0 * e"),
}


def _mutant(tmp_path, name, old, new):
    src = open(MLP_SRC).read()
    assert old in src, f"mutation {name}: pattern not found"
    path = tmp_path / f"mlp_{name}.py"
    path.write_text(src.replace(old, new, 1))
    spec = importlib.util.spec_from_file_location(f"mlp_{name}", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _failed_pins(M):
    failed = []
    for pin in PINS:
        try:
            with np.errstate(all="ignore"):
                pin(M)
        except AssertionError:
            failed.append(pin.__name__)
    return failed


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    M = _mutant(tmp_path, name, *MUTATIONS[name])
    failed = _failed_pins(M)
    assert failed, f"planted mistake {name} passed every pin"


def test_unmodified_copy_passes(tmp_path):
    src = open(MLP_SRC).read()
    path = tmp_path / "mlp_copy.py"
    path.write_text(src)
    spec = importlib.util.spec_from_file_location("mlp_copy", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    assert _failed_pins(mod) == []
