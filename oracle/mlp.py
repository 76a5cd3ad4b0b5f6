"""FP64 oracle of the learned warm start (an addition to the paper's method).

TEST INFRASTRUCTURE ONLY.  The paper's warm start is the RB solution
(Alg. 5); related work it cites (Sec. 1) uses neural-network initial guesses.
Here a small MLP maps log-scaled parameters to the RB coefficients c(mu):

    x = (log10 mu - m) / s                      (input scaling)
    h_1 = gelu(W_1 x + b_1), ..., h_L = gelu(W_L h_{L-1} + b_L)
    c_hat = W_out h_L + b_out                  (no output activation)
    loss = mean over batch and outputs of (c_hat - c)^2
    gelu(z) = z * Phi(z) = z/2 (1 + erf(z / sqrt 2))   (exact erf form)

Adam (beta1 0.9, beta2 0.999, eps 1e-8) updates FP32 master weights.  All
arithmetic here is float64 numpy; weights are passed in by the caller.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def forward(params: List[Tuple[np.ndarray, np.ndarray]], x: np.ndarray):
    """Returns (output, cache).  params = [(W, b), ...], W of shape (out, in)."""
    h = np.asarray(x, dtype=np.float64)
    cache = []
    L = len(params)
    for li, (W, b) in enumerate(params):
        z = h @ np.asarray(W, np.float64).T + np.asarray(b, np.float64)
        cache.append((h, z))
        h = gelu(z) if li < L - 1 else z
    return h, cache


def mse(out, target) -> float:
    d = out - target
    return float(np.mean(d * d))


def backward(params, cache, out, target):
    """Gradients of the mean-squared loss: list of (dW, db) and dX."""
    B, Nout = out.shape
    g = 2.0 * (out - target) / (B * Nout)          # d loss / d out
    grads = [None] * len(params)
    L = len(params)
    for li in range(L - 1, -1, -1):
        W, _ = params[li]
        h_in, z = cache[li]
        dz = g if li == L - 1 else g * gelu_grad(z)
        grads[li] = (dz.T @ h_in, dz.sum(axis=0))
        g = dz @ np.asarray(W, np.float64)
    return grads, g


def loss_and_grads(params, x, target):
    out, cache = forward(params, x)
    grads, dx = backward(params, cache, out, target)
    return mse(out, target), grads, dx


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), in place; t is the 1-based step."""
    for i, ((W, b), (dW, db)) in enumerate(zip(params, grads)):
        for P, G, M, Vv in ((W, dW, m[i][0], v[i][0]), (b, db, m[i][1], v[i][1])):
            M *= beta1
            M += (1.0 - beta1) * G
            Vv *= beta2
            Vv += (1.0 - beta2) * G * G
            mh = M / (1.0 - beta1 ** t)
            vh = Vv / (1.0 - beta2 ** t)
            P -= lr * mh / (np.sqrt(vh) + eps)


def scale_inputs(mu, log_cols: int, lin_lo=None, lin_hi=None, m=0.0, s=1.0):
    """x = (log10 mu - m)/s on the first log_cols columns; the rest map
    [lin_lo, lin_hi] linearly onto [-1, 1]."""
    mu = np.asarray(mu, np.float64)
    x = np.empty_like(mu)
    x[:, :log_cols] = (np.log10(mu[:, :log_cols]) - m) / s
    if mu.shape[1] > log_cols:
        c = 0.5 * (lin_lo + lin_hi)
        hw = 0.5 * (lin_hi - lin_lo)
        x[:, log_cols:] = (mu[:, log_cols:] - c) / hw
    return x
