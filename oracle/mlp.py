"""FP64 CPU oracle of the learned parameter selector's network (test
infrastructure: only ``tests/`` may use it).

The network is not from the paper: it is the fully connected map
    h1 = tanh(W1 x + b1),  h2 = tanh(W2 h1 + b2),  y = W3 h2 + b3
with 10 inputs, 64 + 64 hidden units and 4 outputs, its mean squared error
    L = sum_i |y(x_i) - t_i|^2 / (4 n),
the gradient of L written out by the chain rule, and one step of Adam
(Kingma and Ba, 2015, Algorithm 1) with bias-corrected moments.  Parameter
vector layout: W1[64][10], b1[64], W2[64][64], b2[64], W3[4][64], b3[4],
row-major with the output index first.

Pins (tests/test_oracle_pins.py): the gradient against central finite
differences of L; Adam's first step against its closed form
theta - lr g / (|g| + eps); forward on weights with a known value.
"""
from __future__ import annotations

import numpy as np

N_IN, N_HID, N_OUT = 10, 64, 4
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAM,)
    out, off = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[off:off + k].reshape(shp)
        off += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(theta, X):
    """Network outputs y [n, 4] for inputs X [n, 10]."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    return h2 @ p["W3"].T + p["b3"]


def loss(theta, X, T):
    r = forward(theta, X) - np.asarray(T, dtype=np.float64)
    return float(np.sum(r * r) / r.size)


def loss_grad(theta, X, T):
    """(L, dL/dtheta) by backpropagation."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    h1 = np.tanh(X @ p["W1"].T + p["b1"])
    h2 = np.tanh(h1 @ p["W2"].T + p["b2"])
    y = h2 @ p["W3"].T + p["b3"]
    r = y - T
    L = float(np.sum(r * r) / r.size)
    e3 = 2.0 * r / r.size                   # dL/dy
    g = {"W3": e3.T @ h2, "b3": e3.sum(axis=0)}
    e2 = (e3 @ p["W3"]) * (1.0 - h2 * h2)   # dL/d(W2 h1 + b2)
    g["W2"] = e2.T @ h1
    g["b2"] = e2.sum(axis=0)
    e1 = (e2 @ p["W2"]) * (1.0 - h1 * h1)   # dL/d(W1 x + b1)
    g["W1"] = e1.T @ X
    g["b1"] = e1.sum(axis=0)
    return L, pack(g)


def adam_step(theta, m, v, g, t, lr, beta1, beta2, eps):
    """One Adam step at step count t >= 1; returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
