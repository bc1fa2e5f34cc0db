"""Pins of the surrogate oracle (oracle/mlp.py) against facts that do not use
its own formulas: finite differences, closed forms of GELU and Adam, and the
hand-expanded one-neuron network."""

import math

import numpy as np
import pytest

from oracle import mlp
from synth import mlp_batch, mlp_init, mlp_shape

SMALL = [5, 7, 6, 4]


def test_gelu_closed_forms():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # GELU(1) = Phi(1)
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    x = np.linspace(-4, 4, 17)
    # Phi(-x) = 1 - Phi(x)  =>  GELU(-x) = GELU(x) - x
    np.testing.assert_allclose(mlp.gelu(-x), mlp.gelu(x) - x, atol=1e-15)
    # large arguments: identity and zero
    assert abs(mlp.gelu(np.array([12.0]))[0] - 12.0) < 1e-12
    assert abs(mlp.gelu(np.array([-12.0]))[0]) < 1e-12


def test_gelu_derivative_finite_difference():
    x = np.linspace(-3, 3, 25)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_deriv(x), fd, atol=1e-8)


def test_one_neuron_network_by_hand():
    sizes = [1, 1, 1]
    w1, b1, w2, b2 = 0.7, -0.2, -1.3, 0.4
    params = np.array([w1, b1, w2, b2])
    for x in (-1.5, 0.0, 0.3, 2.0):
        z = w1 * x + b1
        expect = w2 * 0.5 * z * (1 + math.erf(z / math.sqrt(2))) + b2
        y, _, _ = mlp.forward(params, sizes, np.array([[x]]))
        assert abs(y[0, 0] - expect) < 1e-15


def test_single_affine_layer_is_a_matrix_product():
    sizes = [3, 2]
    rng = np.random.default_rng(0)
    W = rng.standard_normal((2, 3))
    b = rng.standard_normal(2)
    X = rng.standard_normal((4, 3))
    params = np.concatenate([W.ravel(), b])
    y, _, _ = mlp.forward(params, sizes, X)
    for n in range(4):
        for o in range(2):
            assert abs(y[n, o] - (sum(X[n, i] * W[o, i] for i in range(3)) + b[o])) < 1e-14


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    params = mlp_init(SMALL, seed=5).astype(np.float64) + 0.1 * rng.standard_normal(
        sum(a * b + b for a, b in zip(SMALL[:-1], SMALL[1:])))
    X = rng.standard_normal((6, SMALL[0]))
    T = rng.standard_normal((6, SMALL[-1]))
    _, g = mlp.loss_and_grad(params, SMALL, X, T)
    h = 1e-6
    fd = np.empty_like(params)
    for i in range(params.size):
        p1, p2 = params.copy(), params.copy()
        p1[i] += h
        p2[i] -= h
        fd[i] = (mlp.loss(p1, SMALL, X, T) - mlp.loss(p2, SMALL, X, T)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    p = np.array([1.0, 2.0, 3.0, 4.0])
    lr = 0.01
    p1, m, v = mlp.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr)
    # bias-corrected first moments are g and g^2: the step is lr g / (|g| + eps)
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_minimises_a_quadratic():
    c = np.array([0.5, -1.0, 2.0])
    p = np.zeros(3)
    m = v = np.zeros(3)
    for t in range(1, 3001):
        p, m, v = mlp.adam_step(p, p - c, m, v, t, 0.01)
    np.testing.assert_allclose(p, c, atol=1e-3)


def test_features_layout():
    X = mlp.features(np.array([0, 5, 7]), 4, np.array([1.0, math.e ** 5, 0.1]), np.array([0, 1, 1]),
                     np.array([0, 2, 12]), 13)
    assert X.shape == (3, 24)
    # q = 0: sines 0, cosines 1
    np.testing.assert_allclose(X[0, :8], [0, 1, 0, 1, 0, 1, 0, 1], atol=1e-15)
    # q index 5 on a 4 x 4 mesh is (1, 1): qx = qy = pi / 2
    np.testing.assert_allclose(X[1, :8], [1, 0, 1, 0, 0, -1, 0, -1], atol=1e-15)
    assert X[1, 8] == pytest.approx(1.0)
    assert X[0, 8] == 0.0
    np.testing.assert_array_equal(X[:, 9:11], [[1, 0], [0, 1], [0, 1]])
    np.testing.assert_array_equal(X[:, 11:].sum(axis=1), [1, 1, 1])
    assert X[2, 11 + 12] == 1.0


def test_adam_training_lowers_the_loss():
    sizes = mlp_shape(12, width=16, n_out=6)
    p = mlp_init(sizes, seed=3).astype(np.float64)
    X, T = mlp_batch(32, 12, 6, seed=4)
    m = v = np.zeros_like(p)
    l0 = mlp.loss(p, sizes, X, T)
    for t in range(1, 201):
        _, g = mlp.loss_and_grad(p, sizes, X, T)
        p, m, v = mlp.adam_step(p, g, m, v, t, 3e-3)
    assert mlp.loss(p, sizes, X, T) < 0.5 * l0


def test_scale_table_interpolation():
    lam = np.array([10.0, 1.0, 0.1, 1e-3])
    s = 3.0 * lam ** -1.5
    # nodes are reproduced and a power law is exact between them
    for l, v in zip(lam, s):
        assert abs(mlp.scale_interp(l, lam, s) / v - 1) < 1e-14
    for l in (5.0, 0.37, 2e-3):
        assert abs(mlp.scale_interp(l, lam, s) / (3.0 * l ** -1.5) - 1) < 1e-12
    # constant beyond the ends
    assert mlp.scale_interp(100.0, lam, s) == pytest.approx(s[0])
    assert mlp.scale_interp(1e-6, lam, s) == pytest.approx(s[-1])
