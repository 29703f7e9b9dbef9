"""Pins of the oracle's objective (Eq. min_obj2 + Eq. regul) and its gradient."""
import numpy as np
import pytest

from oracle import objective, poisson, simplex


def tiny(seed=0, M=7, N=4, D=9, gamma=0.3):
    rng = np.random.default_rng(seed)
    mu = np.linspace(0, 6, D)
    F = poisson.dense_F(mu, M, 0.0, poisson.TRUNCATE)
    P = rng.random((D, N))
    Pi = simplex.project_rows(rng.normal(size=(M, N)))
    return F, P, Pi, gamma


def test_hand_computed_value():
    # F = I (2x2), P = [[1, 0], [0, 1]], Pi = [[.5, .5], [.5, .5]], gamma = 2
    F = np.eye(2)
    P = np.eye(2)
    Pi = np.full((2, 2), 0.5)
    # residual entries are +-0.5 -> data term 4 * 0.25 = 1; regulariser is 0
    assert objective.objective(F, P, Pi, 2.0) == 1.0
    Pi2 = np.array([[1.0, 0.0], [0.0, 1.0]])
    # data term 0; regulariser 2 * ((1-0)^2 + (0-1)^2) = 4
    assert objective.objective(F, P, Pi2, 2.0) == 4.0


@pytest.mark.parametrize("gamma", [0.0, 0.3, 5.0])
def test_gradient_central_differences(gamma):
    F, P, Pi, _ = tiny(gamma=gamma)
    G = objective.gradient(F, P, Pi, gamma)
    h = 1e-6
    for (i, n) in [(0, 0), (3, 2), (6, 3), (1, 1), (5, 0)]:
        E = np.zeros_like(Pi)
        E[i, n] = h
        fd = (objective.objective(F, P, Pi + E, gamma) - objective.objective(F, P, Pi - E, gamma)) / (2 * h)
        assert fd == pytest.approx(G[i, n], rel=1e-7, abs=1e-9)


def test_noiseless_closed_forms():
    F, _, Pi, gamma = tiny(seed=3)
    P = F @ Pi
    # data term vanishes: f = gamma * sum of squared neighbour differences
    d = np.diff(Pi, axis=0)
    assert objective.objective(F, P, Pi, gamma) == pytest.approx(gamma * np.sum(d * d), rel=1e-14)
    G = objective.gradient(F, P, Pi, gamma)
    # and the gradient is the regulariser's alone, checked by central differences of it
    h = 1e-6
    for (i, n) in [(0, 1), (4, 2), (6, 0)]:
        E = np.zeros_like(Pi)
        E[i, n] = h
        fd = (objective.regulariser(Pi + E, gamma) - objective.regulariser(Pi - E, gamma)) / (2 * h)
        assert G[i, n] == pytest.approx(fd, rel=1e-7, abs=1e-12)
    # gamma = 0: zero objective and zero gradient at the generating POVM
    assert objective.objective(F, P, Pi, 0.0) < 1e-28
    assert np.max(np.abs(objective.gradient(F, P, Pi, 0.0))) < 1e-14


def test_sparse_and_dense_agree():
    mu = np.linspace(0, 300, 120)
    F, lo, hi = poisson.build_F(mu, 256, 1e-16, poisson.LUMP)
    rng = np.random.default_rng(1)
    P = rng.random((120, 5))
    Pi = simplex.project_rows(rng.normal(size=(256, 5)))
    Fd = F.toarray()
    assert objective.objective(F, P, Pi, 0.1) == pytest.approx(objective.objective(Fd, P, Pi, 0.1), rel=1e-14)
    assert np.allclose(objective.gradient(F, P, Pi, 0.1), objective.gradient(Fd, P, Pi, 0.1), rtol=1e-13, atol=1e-15)
