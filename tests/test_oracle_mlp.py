"""Pins of the sizing network oracle: finite differences and Adam closed forms."""
import numpy as np

from oracle import mlp


def test_param_count():
    assert mlp.n_params() == 64 * 32 + 64 + 64 * 64 + 64 + 2 * 64 + 2


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    th = rng.standard_normal(mlp.n_params()) * 0.2
    X = rng.standard_normal((7, 32))
    T = rng.standard_normal((7, 2))
    g = mlp.grad(th, X, T)
    idx = rng.choice(th.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (mlp.loss(th + e, X, T) - mlp.loss(th - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9


def test_forward_is_relu_mlp_by_hand():
    """A 1-sample forward against a hand-expanded two-hidden-layer formula."""
    rng = np.random.default_rng(1)
    th = rng.standard_normal(mlp.n_params())
    x = rng.standard_normal(32)
    (W1, b1), (W2, b2), (W3, b3) = mlp.unpack(th)
    h1 = [max(0.0, sum(W1[o, i] * x[i] for i in range(32)) + b1[o]) for o in range(64)]
    h2 = [max(0.0, sum(W2[o, i] * h1[i] for i in range(64)) + b2[o]) for o in range(64)]
    y = [sum(W3[o, i] * h2[i] for i in range(64)) + b3[o] for o in range(2)]
    out, _ = mlp.forward(th, x[None, :])
    assert np.allclose(out[0], y, rtol=1e-12, atol=1e-12)


def test_adam_first_step_is_signed_lr():
    """First Adam step: m-hat = g, v-hat = g^2, so the update is lr g/(|g|+eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th, m, v = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((64, 32))
    T = np.stack([np.tanh(X[:, 0]), X[:, 1] * 0.5], axis=1)
    th = rng.standard_normal(mlp.n_params()) * 0.1
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0 = mlp.loss(th, X, T)
    for s in range(1, 201):
        th, m, v = mlp.adam_step(th, mlp.grad(th, X, T), m, v, s, 3e-3)
    assert mlp.loss(th, X, T) < 0.2 * l0
