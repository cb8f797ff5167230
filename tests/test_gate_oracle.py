"""Pins of the gate oracle (no GPU): its gradient against central finite differences
of its loss, Adam's first steps against their closed form, GELU against the erf
form and its own finite differences, and special cases of the network."""
import math

import numpy as np
import pytest

from oracle import gate_oracle as G


def _theta(seed=0, scale=0.1):
    rng = np.random.default_rng(seed)
    return rng.normal(scale=scale, size=G.N_PARAMS)


def test_layout_size():
    assert G.N_PARAMS == 65921
    p = G.unpack(np.arange(G.N_PARAMS, dtype=np.float64))
    assert p["W1"][0, 0] == 0 and p["W1"][1, 0] == G.N_IN and p["b3"][0] == G.N_PARAMS - 1


def test_gelu_matches_erf_form_and_its_derivative():
    x = np.linspace(-6, 6, 2001)
    exact = 0.5 * x * (1.0 + np.array([math.erf(v / math.sqrt(2.0)) for v in x]))
    # the tanh form is a published approximation of the erf form, good to a few 1e-4
    assert np.abs(G.gelu(x) - exact).max() < 1e-3
    assert G.gelu(np.array([0.0]))[0] == 0.0
    h = 1e-6
    fd = (G.gelu(x + h) - G.gelu(x - h)) / (2 * h)
    assert np.abs(fd - G.gelu_grad(x)).max() < 1e-8


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    theta = _theta(2)
    X = rng.normal(size=(5, G.N_IN))
    t = rng.normal(size=5)
    y, cache = G.forward(theta, X)
    g = G.backward(theta, cache, y, t)
    idx = np.concatenate([rng.choice(G.N_PARAMS, 60, replace=False),
                          [0, G.N_H * G.N_IN, G.N_PARAMS - 1, G.N_PARAMS - 2]])
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd = (G.loss(G.forward(tp, X)[0], t) - G.loss(G.forward(tm, X)[0], t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, i


def test_zero_weights_give_the_output_bias():
    theta = np.zeros(G.N_PARAMS)
    theta[-1] = 0.75
    y, _ = G.forward(theta, np.random.default_rng(3).normal(size=(4, G.N_IN)))
    assert np.allclose(y, 0.75)


def test_adam_first_steps_closed_form():
    """With bias correction, Adam's first step moves each parameter by
    lr * g / (|g| + eps); with a constant gradient every later step does the same."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    theta = np.zeros(4)
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 1e-3, 1e-8
    for step in (1, 2, 3):
        new, m, v = G.adam(theta, g, m, v, step, lr, eps=eps)
        expect = theta - lr * g / (np.abs(g) + eps)
        assert np.allclose(new, expect, rtol=1e-12, atol=1e-15)
        theta = new


def test_features_layout_and_floor():
    s = np.zeros((G.WINDOW, G.MODES, G.TOPK))
    s[7, 2, 15] = 100.0
    x = G.features(s)
    assert x.shape == (G.N_IN,)
    assert x[-1] == pytest.approx(2.0) and x[0] == pytest.approx(-30.0)


def test_decision_rule():
    sig = np.ones((3, 16))
    ranks = (4, 4, 2)
    assert G.runs_exact_pass(-9.0, 1e-5, 7, sig, ranks, 1e-12)          # short history
    assert G.runs_exact_pass(-5.4, 1e-5, 8, sig, ranks, 1e-12)          # within half a decade
    assert not G.runs_exact_pass(-5.6, 1e-5, 8, sig, ranks, 1e-12)      # far below
    small = sig.copy()
    small[2, 1] = 1e-7
    assert G.runs_exact_pass(-9.0, 1e-5, 8, small, ranks, (0.5e-5) ** 2)  # removal candidate
