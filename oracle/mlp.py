"""CPU oracle of the learned cost model: a 6 -> 64 -> 64 -> 1 perceptron
(tanh hidden layers, linear output), its mean-squared-error gradient by
back-propagation and one Adam step, in float64 with numpy.

TEST INFRASTRUCTURE ONLY: the test suite is the only caller.  It shares no
code with the GPU kernels; the parameter layout is the one the library's
C ABI documents: W1[64][6], b1[64], W2[64][64], b2[64], w3[64], b3.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 6, 64
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("w3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    """Named views of a flat parameter vector."""
    p = np.asarray(p, dtype=np.float64)
    out, off = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = p[off:off + k].reshape(shape)
        off += k
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def forward(p, X):
    """y = w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3 for every row x of X."""
    q = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ q["W1"].T + q["b1"])
    h2 = np.tanh(h1 @ q["W2"].T + q["b2"])
    return h2 @ q["w3"] + q["b3"][0]


def loss(p, X, t):
    """Mean squared error (1/m) sum_s (y_s - t_s)^2."""
    return float(np.mean((forward(p, X) - np.asarray(t, dtype=np.float64)) ** 2))


def loss_grad(p, X, t):
    """(loss, gradient) by back-propagation through the two tanh layers:
    dL/dy_s = 2 (y_s - t_s) / m; a tanh unit passes back (1 - h^2) times the
    gradient it receives; each weight collects input x its unit's delta."""
    q = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    m = X.shape[0]
    h1 = np.tanh(X @ q["W1"].T + q["b1"])
    h2 = np.tanh(h1 @ q["W2"].T + q["b2"])
    y = h2 @ q["w3"] + q["b3"][0]
    g = 2.0 * (y - t) / m                      # dL/dy
    d2 = (g[:, None] * q["w3"][None, :]) * (1.0 - h2 ** 2)   # dL/dz2
    d1 = (d2 @ q["W2"]) * (1.0 - h1 ** 2)                    # dL/dz1
    grad = {
        "W1": d1.T @ X, "b1": d1.sum(axis=0),
        "W2": d2.T @ h1, "b2": d2.sum(axis=0),
        "w3": h2.T @ g, "b3": np.array([g.sum()]),
    }
    return float(np.mean((y - t) ** 2)), pack(grad)


def adam_step(p, grad, m1, m2, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, 2015): moment estimates, their bias
    corrections for step number ``step`` (>= 1), and the update."""
    m1 = beta1 * m1 + (1.0 - beta1) * grad
    m2 = beta2 * m2 + (1.0 - beta2) * grad * grad
    mh = m1 / (1.0 - beta1 ** step)
    vh = m2 / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m1, m2


def init(seed: int = 0) -> np.ndarray:
    """Seeded initial parameters (uniform +-1/sqrt(fan-in), zero biases)."""
    rng = np.random.default_rng(seed)
    return pack({
        "W1": rng.uniform(-1, 1, (N_H, N_IN)) / np.sqrt(N_IN), "b1": np.zeros(N_H),
        "W2": rng.uniform(-1, 1, (N_H, N_H)) / np.sqrt(N_H), "b2": np.zeros(N_H),
        "w3": rng.uniform(-1, 1, N_H) / np.sqrt(N_H), "b3": np.zeros(1),
    })
