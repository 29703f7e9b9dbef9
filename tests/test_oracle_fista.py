"""Pins of the oracle's solver (accelerated projected gradient with restart) and certificates."""
import json
import math
import os

import numpy as np
import pytest

from oracle import certify, fista, objective, poisson, simplex
from paper_2404_02844_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def c1():
    inst = synth.c1_small()
    F, lo, hi = poisson.build_F(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    return inst, F


def test_lipschitz_is_the_top_eigenvalue(c1):
    inst, F = c1
    Fd = F.toarray()
    M = inst.M
    Lm = np.diag(np.r_[1.0, np.full(M - 2, 2.0), 1.0]) - np.eye(M, k=1) - np.eye(M, k=-1)
    H = 2 * Fd.T @ Fd + 2 * inst.gamma * Lm
    lam = np.linalg.eigvalsh(H)[-1]
    assert fista.lipschitz(F, inst.gamma, M) == pytest.approx(1.05 * lam, rel=1e-9)


def test_monotone_and_converging(c1):
    inst, F = c1
    L = fista.lipschitz(F, inst.gamma, inst.M)
    r = fista.fista_r(F, inst.P, inst.gamma, L, 600)
    assert np.all(np.diff(r.history) <= 0)
    Xs = r.X
    assert np.all(Xs >= 0) and np.max(np.abs(Xs.sum(1) - 1)) < 1e-14
    k1 = certify.kkt_residual(F, inst.P, fista.fista_r(F, inst.P, inst.gamma, L, 100).X, inst.gamma)
    k2 = certify.kkt_residual(F, inst.P, Xs, inst.gamma)
    assert k2 < k1


def test_polished_optimum_and_bounds(c1):
    inst, F = c1
    with open(os.path.join(GOLDEN, "c1_oracle.json")) as fh:
        gold = json.load(fh)
    L = fista.lipschitz(F, inst.gamma, inst.M)
    assert L == pytest.approx(gold["L_hat"], rel=1e-13)
    r = fista.fista_r(F, inst.P, inst.gamma, L, 2000)
    assert r.f == pytest.approx(gold["f_2000"], rel=1e-12)
    fstar = gold["f_star"]
    # optimum certified by sign checks of the polished active-set solution
    assert gold["polish_certified"]
    # Frank-Wolfe gap bounds the suboptimality
    assert certify.fw_gap(F, inst.P, r.X, inst.gamma) >= r.f - fstar
    assert r.f >= fstar * (1 - 1e-14)
    # the KKT residual of the polished point is at rounding level
    Xstar = np.array(gold["Pi_star"])
    assert certify.kkt_residual(F, inst.P, Xstar, inst.gamma) < 1e-12
    assert objective.objective(F, inst.P, Xstar, inst.gamma) == pytest.approx(fstar, rel=1e-13)


def test_single_outcome_is_trivial():
    mu = np.linspace(0, 10, 12)
    F = poisson.dense_F(mu, 16, 0.0, poisson.TRUNCATE)
    P = np.ones((12, 1))
    r = fista.fista_r(F, P, 0.1, fista.lipschitz(F, 0.1, 16), 5)
    assert np.array_equal(r.X, np.ones((16, 1)))


def test_vacuum_probe_spreads_by_regulariser():
    # one probe with mu = 0 sees only m = 0; with gamma > 0 every row must equal P_0
    M, N = 12, 4
    F = poisson.dense_F(np.array([0.0]), M, 0.0, poisson.TRUNCATE)
    assert np.array_equal(F[0], np.eye(M)[0])
    P0 = np.array([[0.1, 0.2, 0.3, 0.4]])
    L = fista.lipschitz(F, 1.0, M)
    r = fista.fista_r(F, P0, 1.0, L, 5000)
    assert np.max(np.abs(r.X - P0)) < 1e-8


def test_huge_gamma_objective_prefers_constant_columns():
    # For Pi = 1 c^T the regulariser vanishes and f(c) = ||s c^T - P||^2 with s = F 1, whose
    # minimiser over the simplex is c* = P_S(P^T s / ||s||^2).
    mu = np.linspace(0, 10, 15)
    M, N = 20, 5
    F = poisson.dense_F(mu, M, 0.0, poisson.TRUNCATE)
    rng = np.random.default_rng(5)
    P = simplex.project_rows(rng.random((15, N)))
    s = F @ np.ones(M)
    cstar = simplex.project_simplex(P.T @ s / (s @ s))
    fstar = objective.objective(F, P, np.outer(np.ones(M), cstar), 1e6)
    for _ in range(50):
        c = simplex.project_simplex(rng.normal(size=N))
        assert objective.objective(F, P, np.outer(np.ones(M), c), 1e6) >= fstar - 1e-15


def test_noiseless_recovery_tiny():
    # M=12, N=4 detector, D=40 probes on [0, 12]: Poisson inversion is ill-posed
    # (cond(F) ~ 4e5), so recovery is pinned at the accuracy that conditioning allows.
    M, B = 12, 3
    Pi_true = synth.click_detector_povm(M, B, 0.7)
    mu = np.linspace(0, 12, 40)
    F = poisson.dense_F(mu, M, 0.0, poisson.TRUNCATE)
    P = F @ Pi_true
    L = fista.lipschitz(F, 0.0, M)
    r = fista.fista_r(F, P, 0.0, L, 40000, exact_sums=False)
    assert r.f <= 1e-12 * np.sum(P * P)
    fids = [certify.fidelity(r.X[:, n], Pi_true[:, n]) for n in range(B + 1)]
    assert min(fids) >= 0.998
    assert np.max(np.abs(r.X - Pi_true)) <= 1e-2


def test_fidelity_closed_forms():
    a = np.array([0.1, 0.5, 0.4])
    assert certify.fidelity(a, a) == pytest.approx(1.0, rel=1e-15)
    assert certify.fidelity(a, 3 * a) == pytest.approx(1.0, rel=1e-15)
    assert certify.fidelity(np.array([1.0, 0, 0]), np.array([0, 1.0, 0])) == 0.0
    # two-level case by hand: sqrt(.5*.2)+sqrt(.5*.8) = .3162+.6325; squared / (1*1)
    assert certify.fidelity(np.array([0.5, 0.5]), np.array([0.2, 0.8])) == pytest.approx(
        (math.sqrt(0.1) + math.sqrt(0.4)) ** 2, rel=1e-15)


def test_kkt_detects_a_planted_mistake(c1):
    # moving mass inside a row of the optimum makes the KKT residual jump
    inst, F = c1
    with open(os.path.join(GOLDEN, "c1_oracle.json")) as fh:
        gold = json.load(fh)
    X = np.array(gold["Pi_star"])
    k0 = certify.kkt_residual(F, inst.P, X, inst.gamma)
    Y = X.copy()
    i = 30
    j = int(np.argmax(Y[i]))
    Y[i, j] -= 0.01
    Y[i, (j + 1) % Y.shape[1]] += 0.01
    assert certify.kkt_residual(F, inst.P, Y, inst.gamma) > 1e3 * max(k0, 1e-16)


# --- row-scaled step (Hessian diagonal per row of Pi) --------------------------------

def _band_instance(M=96, seed=3):
    rng = synth.rng_for(90, spawn=seed)
    inst = synth.random_detector(rng, M, bins=(6, 6))
    F, lo, hi = poisson.build_F(inst.mu, inst.M, 1e-16, inst.tail_mode)
    return inst, F


@pytest.mark.parametrize("which", ["c1", "band"])
def test_hessian_diag_is_the_diagonal_of_the_hessian(c1, which):
    inst, F = c1 if which == "c1" else _band_instance()
    M = inst.M
    # column m of the Hessian from its action on the unit vector e_m
    cols = np.stack([fista.hessian_apply(F, inst.gamma, np.eye(M)[m]) for m in range(M)], axis=1)
    h = fista.hessian_diag(F, inst.gamma, M)
    assert np.allclose(h, np.diag(cols), rtol=1e-13, atol=0)
    # positive definite diagonal, largest where few photon numbers share the probes (small m)
    assert np.all(h > 0)


def test_row_weights_floor_and_degenerate():
    F = np.zeros((3, 4))
    assert np.array_equal(fista.row_weights(F, 0.0, 4), np.ones(4))
    F[0, 0] = 1.0  # only row 0 is seen; the others get the floored weight
    w = fista.row_weights(F, 0.0, 4)
    assert w[0] == 0.5 and np.all(w[1:] == 1.0 / (1e-12 * 2.0))


@pytest.mark.parametrize("which", ["c1", "band"])
def test_scaled_lipschitz_is_the_top_eigenvalue(c1, which):
    inst, F = c1 if which == "c1" else _band_instance()
    M = inst.M
    Fd = F.toarray()
    Lm = np.diag(np.r_[1.0, np.full(M - 2, 2.0), 1.0]) - np.eye(M, k=1) - np.eye(M, k=-1)
    H = 2 * Fd.T @ Fd + 2 * inst.gamma * Lm
    w = fista.row_weights(F, inst.gamma, M)
    S = np.sqrt(w)[:, None] * H * np.sqrt(w)[None, :]
    lam = np.linalg.eigvalsh(S)[-1]
    # a diagonal scaling gives the scaled matrix a unit diagonal
    assert np.allclose(np.diag(S), 1.0, rtol=1e-12)
    got = fista.lipschitz_scaled(F, inst.gamma, M, w, iters=400)
    assert got == pytest.approx(1.05 * lam, rel=1e-8)
    # and it conditions the problem better than the plain step
    ev = np.linalg.eigvalsh(H)
    evs = np.linalg.eigvalsh(S)
    assert evs[-1] / evs[0] < ev[-1] / ev[0]


def test_scaled_projected_step_decreases_f():
    # descent lemma in the metric diag(1/w): a step of length w_m / L_w per row from any
    # feasible point never raises f (a wrong square root in L_w breaks this)
    inst, F = _band_instance()
    M, N = inst.M, inst.N
    w = fista.row_weights(F, inst.gamma, M)
    Lw = fista.lipschitz_scaled(F, inst.gamma, M, w)
    rng = np.random.default_rng(11)
    for _ in range(20):
        X = simplex.project_rows(rng.normal(size=(M, N)) * rng.uniform(0.01, 3))
        G = objective.gradient(F, inst.P, X, inst.gamma)
        Xn = simplex.project_rows(X - (w / Lw)[:, None] * G)
        assert objective.objective(F, inst.P, Xn, inst.gamma) <= objective.objective(F, inst.P, X, inst.gamma) * (1 + 1e-14)


def test_scaled_solver_reaches_the_certified_optimum(c1):
    inst, F = c1
    with open(os.path.join(GOLDEN, "c1_oracle.json")) as fh:
        gold = json.load(fh)
    w = fista.row_weights(F, inst.gamma, inst.M)
    Lw = fista.lipschitz_scaled(F, inst.gamma, inst.M, w)
    r = fista.fista_r(F, inst.P, inst.gamma, Lw, 6000, row_w=w)
    assert np.all(np.diff(r.history) <= 0)
    fstar = gold["f_star"]
    assert r.f >= fstar * (1 - 1e-14)
    assert (r.f - fstar) <= 1e-11 * fstar
    assert np.max(np.abs(r.X - np.array(gold["Pi_star"]))) <= 2e-6
    # fewer iterations to a relative objective of 1e-9 than with the uniform step
    L = fista.lipschitz(F, inst.gamma, inst.M)
    plain = fista.fista_r(F, inst.P, inst.gamma, L, 6000, f_star=fstar, rel_tol=1e-9)
    scaled = fista.fista_r(F, inst.P, inst.gamma, Lw, 6000, row_w=w, f_star=fstar, rel_tol=1e-9)
    assert scaled.iters < 0.5 * plain.iters, (scaled.iters, plain.iters)


def test_constant_weights_give_the_plain_iteration(c1):
    inst, F = c1
    L = fista.lipschitz(F, inst.gamma, inst.M)
    a = fista.fista_r(F, inst.P, inst.gamma, L, 200)
    b = fista.fista_r(F, inst.P, inst.gamma, L, 200, row_w=np.ones(inst.M))
    assert np.array_equal(a.X, b.X)


def test_momentum_schedule_hand_computed():
    """Three iterations on a problem small enough to follow by hand: F = I (two probes, two
    photon numbers), gamma = 0, P = [[0.9, 0.1], [0.2, 0.8]], L_hat = 20, from Pi = 1/N.
    The expected values were computed with 40-digit arithmetic straight from the
    definitions -- t_1 = 1, t_{k+1} = (1 + sqrt(1 + 4 t_k^2)) / 2, beta_k = (t_k - 1) /
    t_{k+1}, Y = X_k + beta_k (X_k - X_{k-1}), gradient 2 (Y - P), and the two-outcome
    projection a = clip((y_1 - y_2 + 1) / 2, 0, 1) -- with no code shared with the
    oracle.  Every step is accepted, with beta = 0, 0.28175..., 0.43404...; the schedules
    beta_k = (t_{k+1} - 1) / t_{k+1} and k / (k + 3) move the third iterate by 2.2e-2 and
    2.9e-3."""
    F = np.eye(2)
    P = np.array([[0.9, 0.1], [0.2, 0.8]])
    expected = [
        ([0.54, 0.46, 0.47, 0.53], 0.405),
        ([0.58614312690451154945, 0.41385687309548845055, 0.43539265482161633791, 0.56460734517838366209],
         0.30783167746649231875),
        ([0.63555409630109732847, 0.36444590369890267153, 0.39833442777417700365, 0.60166557222582299635],
         0.21853636244727908016),
    ]
    for k, (X, f) in enumerate(expected, start=1):
        r = fista.fista_r(F, P, 0.0, 20.0, k)
        assert r.rejects == 0 and r.iters == k
        assert np.max(np.abs(r.X.ravel() - np.array(X))) < 1e-14
        assert r.f == pytest.approx(f, rel=1e-14)


def test_fw_gap_closed_forms():
    """With F = I and gamma = 0 the gradient is 2 (Pi - P), which gives the Frank-Wolfe gap
    in closed form: at Pi = 1/N each row contributes 2 (max_n P_in - 1/N) (its inner
    product with the gradient vanishes); at a vertex e_j it contributes 2 (1 - P_ij +
    max_{n != j} P_in); at Pi = P it is zero."""
    rng = np.random.default_rng(11)
    M, N = 7, 5
    P = simplex.project_rows(rng.random((M, N)))
    F = np.eye(M)
    U = np.full((M, N), 1.0 / N)
    assert certify.fw_gap(F, P, U, 0.0) == pytest.approx(2.0 * np.sum(P.max(1) - 1.0 / N), rel=1e-14)
    j = rng.integers(0, N, size=M)
    V = np.zeros((M, N))
    V[np.arange(M), j] = 1.0
    others = np.where(np.arange(N)[None, :] == j[:, None], -np.inf, P).max(1)
    want = 2.0 * np.sum(1.0 - P[np.arange(M), j] + others)
    assert certify.fw_gap(F, P, V, 0.0) == pytest.approx(want, rel=1e-14)
    assert abs(certify.fw_gap(F, P, P, 0.0)) < 1e-15


def test_gradient_restart_hand_computed():
    """The gradient restart on the 2x2 problem above (F = I, gamma = 0, Pi = 1/N start),
    computed with 40-digit arithmetic from the definitions, with the step test
    sum_m (1 / w_m) sum_n (Y - X')(X' - X_k) > 0 after each accepted step.
    (a) P = [[0.9, 0.1], [0.2, 0.8]], L_hat = 3: the third step triggers the reset, so the
        fourth is a plain projected step (beta 0 instead of 0.531...); the function
        restart alone keeps the momentum and lands elsewhere.
    (b) P = [[0.9, 0.1], [0.6, 0.4]], L_hat = 3.5, row weights (1, 0.5): the reset comes
        after the fourth step in the weighted metric (after the third without the 1/w_m
        weights)."""
    F = np.eye(2)
    Pa = np.array([[0.9, 0.1], [0.2, 0.8]])
    want_a = [0.903339154488979523997, 0.0966608455110204760029, 0.197495634133265357002, 0.802504365866734642998]
    r = fista.fista_r(F, Pa, 0.0, 3.0, 4, restart="gradient")
    assert r.rejects == 0
    assert np.max(np.abs(r.X.ravel() - np.array(want_a))) < 1e-14
    assert r.f == pytest.approx(0.000034843602191475331396, rel=1e-12)
    plain = fista.fista_r(F, Pa, 0.0, 3.0, 4)
    want_plain = [0.908546615718376670023, 0.0914533842816233299769, 0.193590038211217497483, 0.806409961788782502517]
    assert np.max(np.abs(plain.X.ravel() - np.array(want_plain))) < 1e-14
    Pb = np.array([[0.9, 0.1], [0.6, 0.4]])
    w = np.array([1.0, 0.5])
    want_b4 = [0.912866395339553487938, 0.0871336046604465120624, 0.590678377762060860622, 0.409321622237939139378]
    want_b5 = [0.905514169431237209116, 0.0944858305687627908839, 0.593341698401472043301, 0.406658301598527956699]
    for k, want in ((4, want_b4), (5, want_b5)):
        r = fista.fista_r(F, Pb, 0.0, 3.5, k, row_w=w, restart="gradient")
        assert np.max(np.abs(r.X.ravel() - np.array(want))) < 1e-14, k
    assert r.f == pytest.approx(0.00014947808938670165948, rel=1e-12)


def test_gradient_restart_reaches_the_certified_optimum(c1):
    inst, F = c1
    with open(os.path.join(GOLDEN, "c1_oracle.json")) as fh:
        gold = json.load(fh)
    w = fista.row_weights(F, inst.gamma, inst.M)
    Lw = fista.lipschitz_scaled(F, inst.gamma, inst.M, w)
    r = fista.fista_r(F, inst.P, inst.gamma, Lw, 20000, exact_sums=False, row_w=w, restart="gradient")
    assert np.all(np.diff(r.history) <= 0)
    assert abs(r.f - gold["f_star"]) <= 1e-12 * gold["f_star"]
    assert np.max(np.abs(r.X - np.array(gold["Pi_star"]))) <= 2e-6
