"""Plain FP64 CPU oracle of the learned error gate.

TEST INFRASTRUCTURE ONLY. Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import this module; the product path never calls
it and shares no code with it.

The gate predicts the base-10 logarithm of the next reconstruction error (the
quantity of eq. (error), Sec. 2.5) from the recent history of the singular values
of the core unfoldings (the quantities of eq. (rot) and eq. (percentage) that drive
rank adaptation), so that the exact error pass can be skipped when the error is
predicted to sit far below the threshold. The paper has no such part; this module
writes out the network, its loss, its gradient and its optimiser from their
textbook definitions, in float64 with no fusion:

* features: 8 consecutive steps x 3 modes x the 16 leading singular values of each
  core unfolding (zero-padded), as log10(max(sigma, 1e-30)), standardised per
  feature with a training-set mean and standard deviation;
* network: 384 -> 128 -> 128 -> 1 fully connected, tanh-form GELU (Hendrycks and
  Gimpel) after each hidden layer, linear output;
* loss: mean squared error over a batch;
* gradient: reverse-mode differentiation of the above, written out by hand;
* optimiser: Adam (Kingma and Ba) with bias correction.

Parameter layout (one flat vector, 65,921 entries): W1 (128 x 384, row-major), b1
(128), W2 (128 x 128), b2 (128), w3 (128), b3 (1).

Parity status: pinned by `-m "not gpu"` tests (central finite differences of the
loss for the gradient, the closed form of Adam's first steps, GELU against the
erf form and its own finite differences, special cases of the network).
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

WINDOW, TOPK, MODES = 8, 16, 3
N_IN = WINDOW * MODES * TOPK          # 384
N_H = 128
N_PARAMS = N_H * N_IN + N_H + N_H * N_H + N_H + N_H + 1   # 65921
SIGMA_FLOOR = 1e-30


def unpack(theta: np.ndarray) -> Dict[str, np.ndarray]:
    """Views of the flat parameter vector in the layout documented above."""
    theta = np.asarray(theta)
    o = 0
    out = {}
    for name, shape in (("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
                        ("w3", (N_H,)), ("b3", (1,))):
        size = int(np.prod(shape))
        out[name] = theta[o:o + size].reshape(shape)
        o += size
    assert o == N_PARAMS
    return out


def gelu(x: np.ndarray) -> np.ndarray:
    """tanh form of the Gaussian error linear unit."""
    c = math.sqrt(2.0 / math.pi)
    return 0.5 * x * (1.0 + np.tanh(c * (x + 0.044715 * x ** 3)))


def gelu_grad(x: np.ndarray) -> np.ndarray:
    """Derivative of `gelu` (product and chain rule)."""
    c = math.sqrt(2.0 / math.pi)
    u = c * (x + 0.044715 * x ** 3)
    t = np.tanh(u)
    du = c * (1.0 + 3.0 * 0.044715 * x ** 2)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * du


def forward(theta: np.ndarray, X: np.ndarray) -> Tuple[np.ndarray, dict]:
    """Network output for each row of X (n x 384), with the intermediates."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = X @ p["W1"].T + p["b1"]
    a1 = gelu(h1)
    h2 = a1 @ p["W2"].T + p["b2"]
    a2 = gelu(h2)
    y = a2 @ p["w3"] + p["b3"][0]
    return y, {"X": X, "h1": h1, "a1": a1, "h2": h2, "a2": a2}


def loss(y: np.ndarray, target: np.ndarray) -> float:
    """Mean squared error."""
    d = np.asarray(y) - np.asarray(target)
    return float(np.mean(d * d))


def backward(theta: np.ndarray, cache: dict, y: np.ndarray, target: np.ndarray) -> np.ndarray:
    """Gradient of `loss` with respect to the flat parameters (same layout)."""
    p = unpack(theta)
    n = y.shape[0]
    dy = 2.0 * (y - target) / n                     # (n,)
    g_w3 = cache["a2"].T @ dy
    g_b3 = np.array([dy.sum()])
    da2 = np.outer(dy, p["w3"])                     # (n, 128)
    dh2 = da2 * gelu_grad(cache["h2"])
    g_W2 = dh2.T @ cache["a1"]
    g_b2 = dh2.sum(axis=0)
    da1 = dh2 @ p["W2"]
    dh1 = da1 * gelu_grad(cache["h1"])
    g_W1 = dh1.T @ cache["X"]
    g_b1 = dh1.sum(axis=0)
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, g_b3])


def adam(theta, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def features(sigma_window: np.ndarray) -> np.ndarray:
    """Raw features of one window: sigma_window[w, n, i] for w = 0..7 (oldest first),
    mode n, singular value i (zero beyond the rank), as log10(max(sigma, 1e-30)),
    flattened with the window index slowest and the value index fastest."""
    s = np.asarray(sigma_window, dtype=np.float64)
    assert s.shape == (WINDOW, MODES, TOPK)
    return np.log10(np.maximum(s, SIGMA_FLOOR)).reshape(-1)


def standardise(x: np.ndarray, mean: np.ndarray, std: np.ndarray) -> np.ndarray:
    return (np.asarray(x) - mean) / std


def runs_exact_pass(yhat: float, eps_th: float, history: int, sigma_last: np.ndarray, ranks, budget: float) -> bool:
    """The decision the gate feeds: the exact error pass runs when the prediction is
    within half a decade of the threshold or above it, when fewer than 8 steps of
    singular values exist since the last reinitialisation, or when some mode could
    drop its last direction within the error budget (the singular-value part of the
    removal test), so that every add and remove decision rests on exact errors."""
    if history < WINDOW:
        return True
    if yhat >= math.log10(eps_th) - 0.5:
        return True
    for n, r in enumerate(ranks):
        s = float(sigma_last[n][r - 1])
        if s * s <= budget:
            return True
    return False
