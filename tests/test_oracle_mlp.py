"""Pins for the FP64 oracle of the learned warm start (an addition to the
paper's Alg. 5 initial value): gradients against central finite
differences, Adam's first step against its closed form, GELU against
textbook values of the normal CDF."""
import math

import numpy as np

from oracle import mlp


def small_net(rng, sizes):
    return [(rng.standard_normal((o, i)) / math.sqrt(i), 0.1 * rng.standard_normal(o))
            for i, o in zip(sizes[:-1], sizes[1:])]


def test_gelu_values():
    assert mlp.gelu(np.array(0.0)) == 0.0
    # Phi(1) = 0.841344746068543, Phi(-1) = 0.158655253931457
    assert abs(mlp.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    assert abs(mlp.gelu(np.array(-1.0)) + 0.15865525393145707) < 1e-15
    assert abs(mlp.gelu(np.array(10.0)) - 10.0) < 1e-12
    z = np.linspace(-4, 4, 17)
    num = (mlp.gelu(z + 1e-6) - mlp.gelu(z - 1e-6)) / 2e-6
    np.testing.assert_allclose(mlp.gelu_grad(z), num, rtol=1e-7, atol=1e-9)


def test_gradients_vs_finite_differences():
    rng = np.random.default_rng(0)
    params = small_net(rng, [3, 16, 16, 5])
    x = rng.standard_normal((7, 3))
    y = rng.standard_normal((7, 5))
    loss, grads, dx = mlp.loss_and_grads(params, x, y)
    eps = 1e-6
    for li, (W, b) in enumerate(params):
        for P, G in ((W, grads[li][0]), (b, grads[li][1])):
            flat = P.reshape(-1)
            g = G.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + eps
                lp = mlp.mse(mlp.forward(params, x)[0], y)
                flat[idx] = old - eps
                lm = mlp.mse(mlp.forward(params, x)[0], y)
                flat[idx] = old
                num = (lp - lm) / (2 * eps)
                assert abs(num - g[idx]) <= 1e-6 * max(1.0, abs(num)) * 10 + 1e-9
    # input gradient too
    for idx in range(3):
        xp, xm = x.copy(), x.copy()
        xp[:, idx] += eps
        xm[:, idx] -= eps
        num = (mlp.mse(mlp.forward(params, xp)[0], y) - mlp.mse(mlp.forward(params, xm)[0], y)) / (2 * eps)
        assert abs(num - dx[:, idx].sum()) <= 1e-7


def test_adam_first_step_closed_form():
    # after one step from m = v = 0 the bias-corrected update is lr*g/(|g|+eps)
    rng = np.random.default_rng(1)
    params = small_net(rng, [2, 4, 3])
    grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params]
    before = [(W.copy(), b.copy()) for W, b in params]
    m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    lr = 1e-3
    mlp.adam_step(params, grads, m, v, 1, lr)
    for (W0, b0), (W1, b1), (gW, gb) in zip(before, params, grads):
        np.testing.assert_allclose(W0 - W1, lr * gW / (np.abs(gW) + 1e-8), rtol=1e-12)
        np.testing.assert_allclose(b0 - b1, lr * gb / (np.abs(gb) + 1e-8), rtol=1e-12)


def test_input_scaling():
    mu = np.array([[0.01, 1.0, 100.0, 0.25], [1.0, 10.0, 0.1, 0.75]])
    x = mlp.scale_inputs(mu, 3, 0.25, 0.75, m=0.0, s=2.0)
    np.testing.assert_allclose(x, [[-1, 0, 1, -1], [0, 0.5, -0.5, 1]], atol=1e-15)
