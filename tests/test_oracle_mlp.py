"""Pins of the cost-model oracle (oracle/mlp.py) against calculus and closed
forms, independent of its own formulas: central finite differences of the
loss, a network whose output is known by hand, and Adam's first step."""
import numpy as np

from oracle import mlp


def _data(m=37, seed=1):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, (m, mlp.N_IN)), rng.normal(size=m)


def test_parameter_count():
    assert mlp.N_PARAMS == 64 * 6 + 64 + 64 * 64 + 64 + 64 + 1 == 4673


def test_gradient_matches_finite_differences():
    """Every parameter class, several entries each: the analytic gradient
    agrees with (L(p + h e) - L(p - h e)) / 2h to the difference's own error."""
    p = mlp.init(3)
    X, t = _data()
    _, g = mlp.loss_grad(p, X, t)
    rng = np.random.default_rng(5)
    idx = np.unique(np.concatenate([rng.integers(0, mlp.N_PARAMS, 60),
                                    [0, 383, 384, 447, 448, 4543, 4544, 4607, 4608, 4671, 4672]]))
    h = 1e-5
    for k in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[k] = h
        fd = (mlp.loss(p + e, X, t) - mlp.loss(p - e, X, t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_forward_closed_form():
    """W1 = 0 makes the hidden layers constant: y = w3 . tanh(W2 tanh(b1) + b2) + b3,
    written out for one hand-picked unit."""
    q = {name: np.zeros(shape) for name, shape in mlp.SIZES}
    q["b1"][0] = 0.5
    q["W2"][3, 0] = 2.0
    q["w3"][3] = -1.5
    q["b3"][0] = 0.25
    p = mlp.pack(q)
    X, _ = _data(5)
    expect = -1.5 * np.tanh(2.0 * np.tanh(0.5)) + 0.25
    assert np.allclose(mlp.forward(p, X), expect, rtol=0, atol=1e-15)
    # a single input feature through one unit of each layer
    q["W1"][0, 2] = 1.0
    p = mlp.pack(q)
    x = X[:, 2]
    assert np.allclose(mlp.forward(p, X), -1.5 * np.tanh(2.0 * np.tanh(x + 0.5)) + 0.25, atol=1e-15)


def test_perfect_fit_has_zero_gradient():
    p = mlp.init(4)
    X, _ = _data(20)
    t = mlp.forward(p, X)
    l, g = mlp.loss_grad(p, X, t)
    assert l == 0.0 and np.all(g == 0.0)


def test_adam_first_step_is_signed_learning_rate():
    """With zero moments and eps = 0, bias correction makes the first step -lr * sign(g)."""
    rng = np.random.default_rng(2)
    p = rng.normal(size=mlp.N_PARAMS)
    g = rng.normal(size=mlp.N_PARAMS)
    z = np.zeros(mlp.N_PARAMS)
    q, m1, m2 = mlp.adam_step(p, g, z, z, 1, lr=0.01, eps=0.0)
    assert np.allclose(q - p, -0.01 * np.sign(g), rtol=1e-9, atol=0)
    assert np.allclose(m1, 0.1 * g) and np.allclose(m2, 0.001 * g * g)


def test_training_reduces_loss():
    """A few hundred full-batch Adam steps fit a smooth target."""
    rng = np.random.default_rng(7)
    X = rng.uniform(-1, 1, (256, mlp.N_IN))
    t = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2]
    p = mlp.init(0)
    m1 = m2 = np.zeros(mlp.N_PARAMS)
    l0 = mlp.loss(p, X, t)
    for k in range(1, 301):
        _, g = mlp.loss_grad(p, X, t)
        p, m1, m2 = mlp.adam_step(p, g, m1, m2, k, lr=3e-3)
    assert mlp.loss(p, X, t) < 0.05 * l0
