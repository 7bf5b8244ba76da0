"""Pins of the oracle's network: modified softplus (Sec. 5, Eq. 22), forward special
cases, finite-difference gradients of the log-radiance loss, and Adam's closed form."""
import json
import math
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(__file__), "golden")
OFF = dict(W1=0, B1=1280, W2=1344, B2=5440, W3=5504, B3=9600, W4=9664, B4=9728)


def test_softplus_mod_closed_forms(O):
    g = json.load(open(os.path.join(GOLD, "paper_constants.json")))["softplus_mod"]
    assert O.softplus_mod(0.0) == pytest.approx(g["value_at_0"], rel=1e-15)
    assert O.softplus_mod_grad(0.0) == g["slope_at_0"]
    assert O.softplus_mod_grad(-1e-12) == pytest.approx(0.5, rel=1e-9)   # C1 at zero
    for z in (-30.0, -3.0, -0.5):
        assert O.softplus_mod(z) == pytest.approx(math.log(1 + math.exp(z)), rel=1e-14)
        assert O.softplus_mod_grad(z) == pytest.approx(1 / (1 + math.exp(-z)), rel=1e-14)
    for z in (0.25, 3.0, 100.0):
        assert O.softplus_mod(z) == pytest.approx(0.5 * z + math.log(2), rel=1e-15)
        assert O.softplus_mod_grad(z) == 0.5


def test_param_count():
    assert 20 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 9729


def test_forward_bias_only(O):
    P = np.zeros(9729)
    P[OFF["B4"]] = -1.3
    y, z = O.mlp_forward(P, np.random.default_rng(0).normal(size=(5, 20)))
    assert np.all(z == -1.3) and np.allclose(y, math.log1p(math.exp(-1.3)), rtol=1e-15)


def test_forward_single_path_network(O):
    # one active unit per layer: z = w4 * relu(w3 * relu(w2 * relu(w1 * x_k + b1) + b2) + b3) + b4
    P = np.zeros(9729)
    k = 7
    P[OFF["W1"] + 20 * 5 + k] = 2.0   # unit 5 of layer 1 reads input k
    P[OFF["B1"] + 5] = -0.5
    P[OFF["W2"] + 64 * 9 + 5] = 1.5   # unit 9 of layer 2 reads unit 5
    P[OFF["W3"] + 64 * 63 + 9] = -0.75
    P[OFF["B3"] + 63] = 2.0
    P[OFF["W4"] + 63] = 0.5
    P[OFF["B4"]] = 0.1
    x = np.zeros((4, 20))
    x[:, k] = [-1.0, 0.2, 1.0, 3.0]
    relu = lambda v: np.maximum(v, 0)
    expect = 0.5 * relu(-0.75 * relu(1.5 * relu(2.0 * x[:, k] - 0.5)) + 2.0) + 0.1
    y, z = O.mlp_forward(P, x)
    assert np.allclose(z, expect, rtol=1e-15)
    assert np.allclose(y, [O.softplus_mod(v) for v in expect], rtol=1e-15)


def test_gradient_finite_differences(O):
    rng = np.random.default_rng(1)
    P = rng.normal(0, 0.4, size=9729)
    x = rng.normal(size=(6, 20))
    tgt = rng.uniform(0.0, 3.0, size=6)
    loss, g = O.mlp_loss_grad(P, x, tgt, 0.01)
    assert loss > 0
    # relative check on a random subset of coordinates, central differences in FP64
    idx = np.concatenate([rng.choice(9729, 150, replace=False), [9728, 9664, 1280, 0]])
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        num = (O.mlp_loss_grad(Pp, x, tgt, 0.01)[0] - O.mlp_loss_grad(Pm, x, tgt, 0.01)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, i


def test_loss_value_definition(O):
    P = np.zeros(9729)
    P[OFF["B4"]] = 0.0  # y = ln 2 for every row
    tgt = np.array([0.0, 1.0, 5.0])
    loss, _ = O.mlp_loss_grad(P, np.zeros((3, 20)), tgt, 0.01)
    expect = np.mean((math.log(math.log(2) + 0.01) - np.log(tgt + 0.01)) ** 2)
    assert loss == pytest.approx(expect, rel=1e-14)


def test_adam_closed_form(O):
    # constant gradient: m_hat = g, v_hat = g^2 at every step -> w moves by lr * g / (|g| + eps)
    rng = np.random.default_rng(2)
    g = rng.normal(size=50)
    w = rng.normal(size=50)
    w0 = w.copy()
    m, v = np.zeros(50), np.zeros(50)
    lr, eps = 5e-3, 1e-8
    for step in range(1, 11):
        O.adam(w, m, v, g, step, lr, 0.9, 0.999, eps)
        expect = w0 - step * lr * g / (np.abs(g) + eps)
        assert np.allclose(w, expect, rtol=1e-12, atol=1e-15)
