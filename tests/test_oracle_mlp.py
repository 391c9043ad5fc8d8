"""Pins for the oracle's GELU network (finite differences, identities, closed forms)."""
import math

import numpy as np

from oracle import mlp


def test_gelu_identities_and_derivative():
    x = np.linspace(-6, 6, 241)
    assert np.allclose(mlp.gelu(x) - mlp.gelu(-x), x, rtol=0, atol=1e-15)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(x), fd, rtol=0, atol=1e-8)
    # standard-normal CDF at 1 times 1: GELU(1) = Phi(1)
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15


def test_backward_against_finite_differences():
    rng = np.random.default_rng(0)
    params = mlp.init_params([5, 7, 6, 4], rng)
    params = [(W, rng.standard_normal(b.shape) * 0.1) for W, b in params]
    X = rng.standard_normal((9, 5))
    T = rng.standard_normal((9, 4))
    Y, cache = mlp.forward(params, X)
    grads = mlp.backward(params, cache, Y, T)
    h = 1e-6
    for li in range(len(params)):
        for which in (0, 1):
            arr = params[li][which]
            g = grads[li][which]
            it = np.nditer(arr, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = arr[idx]
                arr[idx] = old + h
                lp = mlp.loss(mlp.forward(params, X)[0], T)
                arr[idx] = old - h
                lm = mlp.loss(mlp.forward(params, X)[0], T)
                arr[idx] = old
                assert abs((lp - lm) / (2 * h) - g[idx]) <= 1e-6 * max(1.0, abs(g[idx]))


def test_single_linear_layer_closed_form():
    rng = np.random.default_rng(1)
    W = rng.standard_normal((3, 4))
    b = rng.standard_normal(3)
    X = rng.standard_normal((6, 4))
    T = rng.standard_normal((6, 3))
    Y, cache = mlp.forward([(W, b)], X)
    assert np.allclose(Y, X @ W.T + b)
    dY = 2 * (Y - T) / Y.size
    (gW, gb), = mlp.backward([(W, b)], cache, Y, T)
    assert np.allclose(gW, dY.T @ X) and np.allclose(gb, dY.sum(0))


def test_adam_step_definition():
    p = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    g = [(np.array([[0.1, 0.2]]), np.array([-0.3]))]
    z = [(np.zeros((1, 2)), np.zeros(1))]
    newp, m, v = mlp.adam_step(p, g, z, z, 1, 0.01)
    # first step: m_hat = g, v_hat = g^2, update = lr * g / (|g| + eps) ~ lr * sign(g)
    assert np.allclose(newp[0][0], [[1.0 - 0.01, -2.0 - 0.01]], atol=1e-9)
    assert np.allclose(newp[0][1], [0.5 + 0.01], atol=1e-9)
    assert np.allclose(m[0][0], 0.1 * np.array([[0.1, 0.2]]))
    assert np.allclose(v[0][0], 0.001 * np.array([[0.01, 0.04]]))


def test_weight_decay_alone_shrinks_weights_only():
    """Decoupled weight decay with a zero gradient: the Adam part is 0, the
    weights shrink by exactly (1 - lr wd), the biases do not move."""
    rng = np.random.default_rng(4)
    p = [(rng.standard_normal((3, 4)), rng.standard_normal(3)), (rng.standard_normal((2, 3)), rng.standard_normal(2))]
    g = [(np.zeros_like(W), np.zeros_like(b)) for W, b in p]
    newp, _, _ = mlp.adam_step(p, g, g, g, 1, 0.05, weight_decay=0.2)
    for (W, b), (W1, b1) in zip(p, newp):
        assert np.array_equal(W1, W - 0.05 * (0.0 + 0.2 * W))
        assert np.allclose(W1, W * (1 - 0.01), rtol=1e-15)
        assert np.array_equal(b1, b)


def test_he_init_scale():
    rng = np.random.default_rng(2)
    W, b = mlp.init_params([400, 300], rng)[0]
    assert abs(W.std() - math.sqrt(2 / 400)) < 0.01 * math.sqrt(2 / 400) * 3
    assert not b.any()
