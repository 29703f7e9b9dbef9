"""Pins of the oracle's two-stage two-metric projected Newton method (App. B).

Each building block against an independent construction on tiny dense problems: the CG
solve against numpy.linalg.solve of the explicit two-metric matrix, the reduced-variable
maps against an explicit T, the reduced Hessian against T^T H T, the line-search slopes
against finite differences; and the whole method against the certified optimum of the
M=64 problem."""
import json
import os

import numpy as np
import pytest

from oracle import fista, newton, objective, poisson, simplex
from paper_2404_02844_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny(M=10, N=4, D=14, gamma=0.05, seed=0):
    mu = np.linspace(0.0, 12.0, D)
    F = poisson.dense_F(mu, M, 0.0, poisson.TRUNCATE)
    rng = np.random.default_rng(seed)
    P = simplex.project_rows(rng.random((D, N)))
    return F, P, gamma


def dense_hessian(F, gamma):
    M = F.shape[1]
    return np.stack([fista.hessian_apply(F, gamma, np.eye(M)[m]) for m in range(M)], axis=1)


def test_pcg_solves_an_spd_system():
    rng = np.random.default_rng(1)
    A = rng.normal(size=(12, 12))
    A = A @ A.T + 12 * np.eye(12)
    b = rng.normal(size=12)
    x, it = newton.pcg(lambda v: A @ v, b, np.diag(A).copy(), 1e-13, 100)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    assert it <= 12 + 1


def test_stage1_direction_solves_the_two_metric_system():
    F, P, gamma = tiny()
    M, N = F.shape[1], P.shape[1]
    rng = np.random.default_rng(2)
    X = simplex.project_rows(rng.normal(size=(M, N)))
    g = objective.gradient(F, P, X, gamma)
    h = fista.hessian_diag(F, gamma, M)
    eps = 1e-12
    D, it, bind = newton.stage1_direction(F, gamma, X, g, h, eps, 1e-14, 500)
    assert bind.any() and (~bind).any()
    # explicit D: column n of Pi couples only with column n; flatten column-major blocks
    A = dense_hessian(F, gamma)
    Dfull = np.zeros((M * N, M * N))
    idx = lambda i, n: n * M + i  # noqa: E731
    for n in range(N):
        for i in range(M):
            for j in range(M):
                if bind[i, n] or bind[j, n]:
                    if i == j:
                        Dfull[idx(i, n), idx(i, n)] = A[i, i]
                else:
                    Dfull[idx(i, n), idx(j, n)] = A[i, j]
    rhs = -g.T.reshape(-1)
    ref = np.linalg.solve(Dfull, rhs).reshape(N, M).T
    assert np.max(np.abs(D - ref)) <= 1e-8 * np.max(np.abs(ref))


def test_reduced_maps_are_adjoint_and_keep_row_sums():
    rng = np.random.default_rng(3)
    M, N = 7, 5
    Pi = simplex.project_rows(rng.normal(size=(M, N)))
    mi = newton.reduce_max(Pi)
    assert np.array_equal(mi, np.array([int(np.flatnonzero(r == r.max())[0]) for r in Pi]))
    v = rng.normal(size=(M, N))
    v[np.arange(M), mi] = 0.0
    w = rng.normal(size=(M, N))
    Tv = newton.expand(v, mi)
    assert np.allclose(Tv.sum(axis=1), 0.0, atol=1e-15)
    assert np.sum(Tv * w) == pytest.approx(np.sum(v * newton.contract(w, mi)), rel=1e-13)
    # explicit T for one row: reduced coordinates n != m(i) -> full row
    i = 2
    keep = [n for n in range(N) if n != mi[i]]
    T = np.zeros((N, N - 1))
    for k, n in enumerate(keep):
        T[n, k] = 1.0
        T[mi[i], k] = -1.0
    assert np.allclose(Tv[i], T @ v[i, keep], atol=1e-15)
    assert np.allclose(newton.contract(w, mi)[i, keep], T.T @ w[i], atol=1e-15)


def test_reduced_hessian_is_TtHT():
    F, P, gamma = tiny(M=6, N=3, D=9)
    M, N = F.shape[1], P.shape[1]
    rng = np.random.default_rng(4)
    X = simplex.project_rows(rng.normal(size=(M, N)))
    mi = newton.reduce_max(X)
    A = dense_hessian(F, gamma)
    H = np.kron(np.eye(N), A)  # column-major flattening: block n = column n
    idx = lambda i, n: n * M + i  # noqa: E731
    red = [(i, n) for i in range(M) for n in range(N) if n != mi[i]]
    T = np.zeros((M * N, len(red)))
    for k, (i, n) in enumerate(red):
        T[idx(i, n), k] = 1.0
        T[idx(i, mi[i]), k] = -1.0
    Hr = T.T @ H @ T
    v = rng.normal(size=(M, N))
    v[np.arange(M), mi] = 0.0
    got = newton.contract(fista.hessian_apply(F, gamma, newton.expand(v, mi)), mi)
    ref = Hr @ np.array([v[i, n] for i, n in red])
    assert np.allclose(np.array([got[i, n] for i, n in red]), ref, rtol=1e-12, atol=1e-14)
    # its diagonal is twice the Hessian diagonal of the row
    h = fista.hessian_diag(F, gamma, M)
    assert np.allclose(np.diag(Hr), [2 * h[i] for i, n in red], rtol=1e-12)


@pytest.mark.parametrize("stage", [1, 2])
def test_slopes_match_finite_differences(stage):
    F, P, gamma = tiny(seed=5)
    M, N = F.shape[1], P.shape[1]
    rng = np.random.default_rng(6)
    X = simplex.project_rows(rng.normal(size=(M, N)) * 0.3)
    g = objective.gradient(F, P, X, gamma)
    h = fista.hessian_diag(F, gamma, M)
    if stage == 1:
        D, _, _ = newton.stage1_direction(F, gamma, X, g, h, 1e-12, 1e-10, 200)
        slope = newton.stage1_slope(X, D, g)
        phi = lambda a: objective.objective(F, P, simplex.project_rows(X + a * D), gamma)  # noqa: E731
    else:
        D, _, mi, _ = newton.stage2_direction(F, gamma, X, g, h, 1e-12, 1e-10, 200)
        slope = newton.stage2_slope(X, D, g, mi)
        phi = lambda a: objective.objective(F, P, newton.stage2_trial(X, D, mi, a), gamma)  # noqa: E731
    a = 1e-6
    fd = (phi(a) - phi(0.0)) / a
    assert slope < 0  # a descent direction
    assert fd == pytest.approx(slope, rel=1e-3, abs=1e-12)


def test_two_stage_reaches_the_certified_optimum():
    inst = synth.c1_small()
    F, _, _ = poisson.build_F(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    with open(os.path.join(GOLDEN, "c1_oracle.json")) as fh:
        gold = json.load(fh)
    fstar = gold["f_star"]
    r = newton.two_stage(F, inst.P, inst.gamma, max_newton=200, eps_kkt=1e-13)
    assert r.stage1_iters >= 1 and r.stage2_iters >= 1
    assert np.all(np.diff(r.history) <= 0)  # Armijo keeps every accepted step monotone
    assert (r.f - fstar) <= 1e-8 * fstar and r.f >= fstar * (1 - 1e-14)
    assert np.max(np.abs(r.X - np.array(gold["Pi_star"]))) <= 1e-4
    assert np.all(r.X >= 0) and np.max(np.abs(r.X.sum(axis=1) - 1)) <= 1e-13


def test_stage2_only_reaches_the_same_optimum():
    inst = synth.c1_small()
    F, _, _ = poisson.build_F(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    with open(os.path.join(GOLDEN, "c1_oracle.json")) as fh:
        fstar = json.load(fh)["f_star"]
    r = newton.two_stage(F, inst.P, inst.gamma, max_newton=300, eps_kkt=1e-13, stage2_only=True)
    assert r.stage1_iters == 0 and r.stage2_iters >= 1
    assert np.all(np.diff(r.history) <= 0)
    assert (r.f - fstar) <= 1e-7 * fstar


def test_tangent_direction_of_the_projected_path():
    # interior row: the derivative is d minus its mean (closed form)
    x = np.array([0.2, 0.3, 0.5])
    d = np.array([1.0, -2.0, 4.0])
    assert np.allclose(newton.tangent_direction(x, d), d - d.mean(), rtol=0, atol=1e-15)
    # hand case with zeros: support {0, 1}; zero entries with d = 3 and -5.
    # t solves (1 - t) + (2 - t) + max(3 - t, 0) = 0  ->  t = 2, entry 2 enters with 1
    x = np.array([0.6, 0.4, 0.0, 0.0])
    d = np.array([1.0, 2.0, 3.0, -5.0])
    assert np.allclose(newton.tangent_direction(x, d), [-1.0, 0.0, 1.0, 0.0], rtol=0, atol=1e-15)
    # random rows with exact zeros against a small-step difference of the projection
    rng = np.random.default_rng(7)
    for _ in range(50):
        x = simplex.project_rows(rng.normal(size=(1, 12)) * 2.0)[0]
        d = rng.normal(size=12)
        v = newton.tangent_direction(x, d)
        a = 1e-7
        fd = (simplex.project_rows((x + a * d)[None, :])[0] - x) / a
        assert np.max(np.abs(v - fd)) <= 1e-6 * max(1.0, np.max(np.abs(v)))
        assert abs(v.sum()) <= 1e-13 and np.all(v[x == 0.0] >= 0.0)
