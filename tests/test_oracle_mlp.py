"""Pins of the oracle's warm-start network: GELU closed forms, central differences of the
backward pass, interpolation exactness, Adam's first step."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_closed_forms():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # far from zero the tanh saturates: gelu(x) -> x for x >> 0 and -> 0 for x << 0
    assert mlp.gelu(np.array([20.0]))[0] == pytest.approx(20.0, rel=1e-15)
    assert abs(mlp.gelu(np.array([-20.0]))[0]) < 1e-15
    # gelu(1) by hand: u = sqrt(2/pi) * 1.044715
    u = math.sqrt(2 / math.pi) * 1.044715
    assert mlp.gelu(np.array([1.0]))[0] == pytest.approx(0.5 * (1 + math.tanh(u)), rel=1e-15)
    x = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(x))) < 1e-9


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    sizes = [7, 6, 5, 4, 9]
    params = mlp.init_params(rng, sizes)
    params = [(W, rng.normal(size=b.shape) * 0.1) for W, b in params]
    X = rng.normal(size=(3, 7))
    T = rng.normal(size=(3, 9))
    out, cache = mlp.forward(params, X)
    loss, dout = mlp.mse(out, T)
    grads = mlp.backward(params, cache, dout)
    h = 1e-6
    for li in range(4):
        for which in (0, 1):
            P = params[li][which]
            G = grads[li][which]
            flat = P.reshape(-1)
            for idx in list(range(min(flat.size, 5))) + [flat.size - 1]:
                orig = flat[idx]
                flat[idx] = orig + h
                lp = mlp.mse(mlp.forward(params, X)[0], T)[0]
                flat[idx] = orig - h
                lm = mlp.mse(mlp.forward(params, X)[0], T)[0]
                flat[idx] = orig
                fd = (lp - lm) / (2 * h)
                assert G.reshape(-1)[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_features_interpolate_exactly_on_linear_columns():
    mu = np.linspace(3.0, 500.0, 77)
    P = np.stack([0.1 + 0.001 * mu, 0.9 - 0.001 * mu, np.zeros_like(mu)], axis=1)
    X = mlp.features(mu, P, bins=2)
    g = mlp.resample_grid(mu)
    assert g[0] == 3.0 and g[-1] == 500.0 and len(g) == 256
    assert np.allclose(X[0, :256], 0.1 + 0.001 * g, atol=1e-15)
    assert np.allclose(X[1, :256], 0.9 - 0.001 * g, atol=1e-15)
    assert X[1, 256] == 0.5 and X[2, 256] == 1.0 and X[0, 257] == 2 / 128


def test_adam_first_step_is_signed_lr():
    # with bias correction, the first Adam step moves every weight by lr * g / (|g| + eps')
    params = [(np.ones((2, 2)), np.zeros(2))]
    grads = [(np.array([[0.5, -2.0], [1e-3, 3.0]]), np.array([1.0, -1.0]))]
    out = mlp.adam_step(params, grads, {}, lr=0.01)
    assert np.allclose(out[0][0], 1.0 - 0.01 * np.sign(grads[0][0]), atol=1e-6)
    assert np.allclose(out[0][1], -0.01 * np.sign(grads[0][1]), atol=1e-7)
