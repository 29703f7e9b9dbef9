"""Warm-start network, FP64 (test infrastructure; the GPU path has its own kernels).

The learned warm start maps the measured statistics of one detector outcome to that
outcome's column of Pi; the solver then starts from the row-wise simplex projection
(Eq. Mp1_proj) of the assembled columns instead of Pi = 1/N (Algorithm 1's start).

Features of outcome n of a detector with B bins and probes mu_0 <= ... <= mu_{D-1}:
    x = [P(g_0; n), ..., P(g_{255}; n), n / B, B / 128]
where P(g; n) linearly interpolates the column P[:, n] on the probe grid at the 256
points g_j = mu_0 + j (mu_{D-1} - mu_0) / 255.

Network: four linear layers 258 -> H -> H -> H -> M (H = 512) with the tanh form of GELU
(Hendrycks and Gimpel 2016),
    gelu(x) = x/2 (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))),
after the first three.  Weights W_l are [out, in]; a layer computes y = x W_l^T + b_l.
Loss: mean of squared errors against the solver's Pi* column; Adam (Kingma and Ba 2015).
"""
from __future__ import annotations

import math

import numpy as np

SQRT_2_OVER_PI = math.sqrt(2.0 / math.pi)
N_GRID = 256


def gelu(x: np.ndarray) -> np.ndarray:
    return 0.5 * x * (1.0 + np.tanh(SQRT_2_OVER_PI * (x + 0.044715 * x ** 3)))


def gelu_grad(x: np.ndarray) -> np.ndarray:
    u = SQRT_2_OVER_PI * (x + 0.044715 * x ** 3)
    t = np.tanh(u)
    du = SQRT_2_OVER_PI * (1.0 + 3.0 * 0.044715 * x ** 2)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * du


def resample_grid(mu: np.ndarray, n_points: int = N_GRID) -> np.ndarray:
    mu = np.asarray(mu, dtype=np.float64)
    return mu[0] + (mu[-1] - mu[0]) * np.arange(n_points) / (n_points - 1)


def features(mu: np.ndarray, P: np.ndarray, bins: int, n_points: int = N_GRID) -> np.ndarray:
    """[B + 1, n_points + 2] feature rows of the detector's real outcomes 0..B."""
    g = resample_grid(mu, n_points)
    rows = []
    for n in range(bins + 1):
        r = np.interp(g, mu, P[:, n])
        rows.append(np.concatenate([r, [n / bins, bins / 128.0]]))
    return np.array(rows)


def init_params(rng: np.random.Generator, sizes) -> list:
    """[(W, b), ...] with W ~ N(0, 1/fan_in) and zero biases."""
    params = []
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        params.append((rng.normal(0.0, 1.0 / math.sqrt(fin), size=(fout, fin)), np.zeros(fout)))
    return params


def forward(params, X: np.ndarray):
    """Returns the output and the cache (layer inputs and pre-activations)."""
    cache = []
    h = np.asarray(X, dtype=np.float64)
    for li, (W, b) in enumerate(params):
        z = h @ W.T + b
        cache.append((h, z))
        h = gelu(z) if li < len(params) - 1 else z
    return h, cache


def backward(params, cache, dout: np.ndarray):
    """Gradients [(dW, db), ...] of a scalar whose derivative w.r.t. the output is dout."""
    grads = [None] * len(params)
    g = dout
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        h, z = cache[li]
        if li < len(params) - 1:
            g = g * gelu_grad(z)
        grads[li] = (g.T @ h, g.sum(axis=0))
        g = g @ W
    return grads


def mse(out: np.ndarray, target: np.ndarray):
    """mean((out - target)^2) and its derivative w.r.t. out."""
    diff = out - target
    n = diff.size
    return float(np.sum(diff * diff) / n), 2.0 * diff / n


def adam_step(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update; state = {"t": int, "m": [...], "v": [...]} (created if empty)."""
    if not state:
        state["t"] = 0
        state["m"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        state["v"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    state["t"] += 1
    t = state["t"]
    out = []
    for k, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, g) in enumerate(((W, gW), (b, gb))):
            m = b1 * state["m"][k][j] + (1 - b1) * g
            v = b2 * state["v"][k][j] + (1 - b2) * g * g
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
            state["m"][k] = (m, state["m"][k][1]) if j == 0 else (state["m"][k][0], m)
            state["v"][k] = (v, state["v"][k][1]) if j == 0 else (state["v"][k][0], v)
        out.append(tuple(new))
    return out
