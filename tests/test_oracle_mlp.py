"""Pins for the FP64 oracle of the learned warm start (an addition to the
paper's Alg. 5 initial value): gradients against central finite
differences, Adam's first step and several steps against the closed form of
its unrolled moment sums, GELU against textbook values of the normal CDF."""
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


def adam_unrolled(theta0, gs, lr, b1, b2, eps=1e-8):
    """Adam's iterate after len(gs) steps from m = v = 0, from the unrolled sums
    m_t = (1 - b1) sum_i b1^(t-i) g_i and v_t = (1 - b2) sum_i b2^(t-i) g_i^2,
    each step lr (m_t / (1 - b1^t)) / (sqrt(v_t / (1 - b2^t)) + eps)."""
    theta = theta0
    for t in range(1, len(gs) + 1):
        m = (1 - b1) * math.fsum(b1 ** (t - i) * gs[i - 1] for i in range(1, t + 1))
        v = (1 - b2) * math.fsum(b2 ** (t - i) * gs[i - 1] ** 2 for i in range(1, t + 1))
        theta -= lr * (m / (1 - b1 ** t)) / (math.sqrt(v / (1 - b2 ** t)) + eps)
    return theta


def test_adam_several_steps_closed_form():
    """Four steps with gradients of changing sign and size, for the default and
    for clearly different (beta1, beta2): swapped betas, a bias correction with
    the wrong exponent or a missing square on v all move the iterate."""
    gs = [1.0, -2.0, 3.0, 0.5]
    # hand value of the third step with the defaults: m3/(1-0.9^3) = 0.201/0.271,
    # v3/(1-0.999^3) = 0.013994001/0.002997001
    step3 = 1e-3 * (0.201 / 0.271) / (math.sqrt(0.013994001 / 0.002997001) + 1e-8)
    assert abs(step3 - 1e-3 * 0.34324108) < 1e-11
    for b1, b2 in ((0.9, 0.999), (0.8, 0.95), (0.5, 0.7)):
        W = np.array([[0.25, -1.5]])
        b = np.array([0.75])
        params = [(W, b)]
        m = [(np.zeros_like(W), np.zeros_like(b))]
        v = [(np.zeros_like(W), np.zeros_like(b))]
        scale = np.array([1.0, -0.5])                # per-entry gradients g_t * scale
        for t, g in enumerate(gs, start=1):
            grads = [(g * scale[None, :], np.array([2.0 * g]))]
            mlp.adam_step(params, grads, m, v, t, 1e-3, beta1=b1, beta2=b2)
        for j, (w0, sc) in enumerate(((0.25, 1.0), (-1.5, -0.5))):
            ref = adam_unrolled(w0, [g * sc for g in gs], 1e-3, b1, b2)
            assert abs(params[0][0][0, j] - ref) <= 1e-14, (b1, b2, j)
        assert abs(params[0][1][0] - adam_unrolled(0.75, [2.0 * g for g in gs], 1e-3, b1, b2)) <= 1e-14
    # the third step on its own (defaults) equals the hand value
    th2 = adam_unrolled(0.0, gs[:2], 1e-3, 0.9, 0.999)
    th3 = adam_unrolled(0.0, gs[:3], 1e-3, 0.9, 0.999)
    assert abs((th2 - th3) - step3) < 1e-15


def test_input_scaling():
    mu = np.array([[0.01, 1.0, 100.0, 0.25], [1.0, 10.0, 0.1, 0.75]])
    x = mlp.scale_inputs(mu, 3, 0.25, 0.75, m=0.0, s=2.0)
    np.testing.assert_allclose(x, [[-1, 0, 1, -1], [0, 0.5, -0.5, 1]], atol=1e-15)
