"""Pins of the oracle's simplex projection (Eq. Mp1_proj) against brute force and closed forms."""
import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st
from hypothesis.extra.numpy import arrays

from oracle import simplex


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 10])
def test_matches_bruteforce(n):
    rng = np.random.default_rng(n)
    for trial in range(40):
        scale = [0.1, 1.0, 10.0][trial % 3]
        x = rng.normal(size=n) * scale
        if trial % 5 == 0:
            x[: n // 2] = x[0]  # ties
        y = simplex.project_simplex(x)
        yb = simplex.project_simplex_bruteforce(x)
        assert np.max(np.abs(y - yb)) < 1e-13


def test_closed_forms():
    # a point of the simplex is its own projection
    p = np.array([0.2, 0.3, 0.5])
    assert np.allclose(simplex.project_simplex(p), p, atol=1e-16)
    # a constant vector goes to the barycentre
    assert np.allclose(simplex.project_simplex(np.full(7, -3.2)), np.full(7, 1 / 7), atol=1e-16)
    # two coordinates: y0 = clip((1 + x0 - x1) / 2, 0, 1)
    for x0, x1 in [(0.3, 0.1), (5.0, -2.0), (-1.0, 0.5), (0.0, 0.0)]:
        y = simplex.project_simplex(np.array([x0, x1]))
        y0 = min(1.0, max(0.0, (1 + x0 - x1) / 2))
        assert y == pytest.approx([y0, 1 - y0], abs=1e-15)
    # one dominant coordinate: the vertex
    assert np.array_equal(simplex.project_simplex(np.array([5.0, 0.1, -1.0])), [1.0, 0.0, 0.0])


vec = arrays(np.float64, st.integers(1, 12), elements=st.floats(-50, 50, allow_nan=False))


@settings(max_examples=200, deadline=None)
@given(vec, st.floats(-10, 10))
def test_properties(x, c):
    y = simplex.project_simplex(x)
    assert np.all(y >= 0)
    assert abs(y.sum() - 1.0) < 1e-12
    # idempotent
    assert np.max(np.abs(simplex.project_simplex(y) - y)) < 1e-12
    # invariant to adding a constant to every coordinate
    assert np.max(np.abs(simplex.project_simplex(x + c) - y)) < 1e-9
    # equivariant under permutations
    perm = np.random.default_rng(len(x)).permutation(len(x))
    assert np.max(np.abs(simplex.project_simplex(x[perm]) - y[perm])) < 1e-12
    # optimality: x - y is constant on the support and >= that constant off it
    g = x - y
    sup = y > 0
    t = g[sup].mean()
    assert np.max(np.abs(g[sup] - t)) < 1e-9
    assert np.all(g[~sup] <= t + 1e-9)


def test_rows_are_independent():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(33, 9))
    Y = simplex.project_rows(X)
    for i in range(33):
        assert np.max(np.abs(Y[i] - simplex.project_simplex_bruteforce(X[i]))) < 1e-13
