"""Pins of the FP64 MLP oracle: finite differences, closed forms, BF16 rounding."""
import math

import numpy as np

from oracle import mlp as M


def _batch(b=3, seed=0):
    rng = np.random.default_rng(seed)
    lam = np.sort(10.0 ** rng.uniform(-8, 0, size=(b, M.NT)), axis=1)[:, ::-1] * 1e6
    z = M.features(lam)
    t = 1.0 / (1.0 + np.exp(-2.0 * (np.arange(1, M.NT + 1)[None, :] - rng.integers(3, 12, size=(b, 1)))))
    c = M.loss_weights(lam, t)
    return lam, z, t, c


def test_gelu_and_sigmoid_values():
    assert abs(M.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15      # Phi(1)
    assert abs(M.gelu(np.array(-1.0)) + 0.15865525393145707) < 1e-15
    assert abs(M.gelu_grad(np.array(0.0)) - 0.5) < 1e-15
    h = np.linspace(-4, 4, 17)
    num = (M.gelu(h + 1e-6) - M.gelu(h - 1e-6)) / 2e-6
    assert np.allclose(M.gelu_grad(h), num, atol=1e-9)


def test_bf16_rounding_ties_to_even():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -2.5, 1.0 + 2.0 ** -7 + 2.0 ** -8], dtype=np.float32)
    got = M.bf16_round(x)
    assert np.array_equal(got, [1.0, 1.0, 1.0 + 2.0 ** -7, -2.5, 1.0 + 2.0 ** -6])


def test_features_normalised_log_spectrum():
    lam = np.array([[100.0, 1.0, 1e-30] + [1e-3] * (M.NT - 3)])
    z = M.features(lam)
    assert z[0, 0] == 0.0 and abs(z[0, 1] + 2.0 / 8.0) < 1e-15
    assert abs(z[0, 2] - math.log10(2.0 ** -52) / 8.0) < 1e-12       # floored at lambda_1 2^-52
    assert M.NPARAM == 131712


def test_backward_matches_central_differences():
    lam, z, t, c = _batch()
    p = M.init_params(3)
    p = {k: v.astype(np.float64) for k, v in p.items()}
    w, cache = M.forward(p, z, bf16=False)
    g = M.backward(cache, t, c)
    rng = np.random.default_rng(1)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in p[name].shape)
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[name][idx] += h
            pm[name][idx] -= h
            lp = M.loss(M.forward(pp, z, bf16=False)[0], t, c)
            lm = M.loss(M.forward(pm, z, bf16=False)[0], t, c)
            num = (lp - lm) / (2 * h)
            assert abs(num - g[name][idx]) <= 1e-6 * max(1.0, abs(num)) + 1e-9, (name, idx, num, g[name][idx])


def test_one_layer_closed_form():
    # W1 = W2 = 0: a2 = GELU(b2) is constant, so w = sigmoid(W3 a2 + b3) and
    # dL/db3 = 2 c (w - t) w (1 - w) / B, dL/dW3 = (dL/db3)^T a2.
    lam, z, t, c = _batch(b=2, seed=4)
    p = {k: np.zeros(s) for k, s in M.SHAPES.items()}
    rng = np.random.default_rng(2)
    p["b2"] = rng.standard_normal(M.H)
    p["W3"] = rng.standard_normal((M.NT, M.H)) * 0.05
    p["b3"] = rng.standard_normal(M.NT)
    w, cache = M.forward(p, z, bf16=False)
    a2 = M.gelu(p["b2"])
    w_ref = 1.0 / (1.0 + np.exp(-(p["W3"] @ a2 + p["b3"])))
    assert np.allclose(w, w_ref[None, :], rtol=1e-14)
    g = M.backward(cache, t, c)
    d3 = 2.0 * c * (w - t) * w * (1.0 - w) / 2.0
    assert np.allclose(g["b3"], d3.sum(0), rtol=1e-12)
    assert np.allclose(g["W3"], np.outer(d3.sum(0), a2), rtol=1e-12)
    assert np.allclose(g["W1"], 0.0) and np.allclose(g["W2"], np.outer(g["b2"], M.gelu(np.zeros(M.H))))


def test_loss_is_relative_energy_error():
    lam, z, t, c = _batch(b=1, seed=5)
    w = t * 1.01
    # first order: sum c (w - t)^2 is the squared relative weight error in the energy metric
    assert abs(M.loss(w, t, c) - 1e-4 * np.sum(lam * t * t) / np.sum(lam * t * t)) < 1e-12


def test_adam_moves_against_gradient():
    p = {k: np.ones(s, dtype=np.float32) for k, s in M.SHAPES.items()}
    g = {k: np.full(s, 0.5) for k, s in M.SHAPES.items()}
    m = {k: np.zeros(s) for k, s in M.SHAPES.items()}
    v = {k: np.zeros(s) for k, s in M.SHAPES.items()}
    M.adam_step(p, g, m, v, 1, 1e-3)
    # first bias-corrected Adam step is lr * sign(g)
    assert np.allclose(p["W1"], 1.0 - 1e-3, atol=1e-7)
