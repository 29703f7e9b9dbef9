"""GPU (HIP, gfx950) vs CPU FP64 oracle, through the C ABI.

Tolerances: FP64 path -- relative objective error <= 1e-9 and max |dPi| <= 1e-6 after
the same number of iterations from the same start with the same step; objective and
gradient evaluations agree to rounding (1e-12 relative).  FP32 path -- 1e-4.
"""
import math

import numpy as np
import pytest

from oracle import certify, fista, objective, poisson, simplex
from paper_2404_02844_amd import _pdt, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pdt.lib()
    return torch.device("cuda:0")


def gpu(a, dev, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=dev).contiguous()


def oracle_F(inst):
    return poisson.build_F(inst.mu, inst.M, inst.threshold, inst.tail_mode)


def small_instance(M=200, B=20, D=300, mu_max=220.0, gamma=1e-3, tail=synth.LUMP, tau=1e-16, seed=7, dark=1e-4):
    return synth.make_instance(f"small_m{M}_b{B}_d{D}", M=M, B=B, eta=0.8, dark=dark, D=D, mu_max=mu_max,
                               shots=1e6, gamma=gamma, tail_mode=tail, threshold=tau, rng=synth.rng_for(90 + seed))


# ---- projection ------------------------------------------------------------------------

@pytest.mark.parametrize("cols", [1, 2, 9, 16, 17, 65, 100, 129, 300, 1024])
def test_projection_matches_oracle(dev, cols):
    rng = np.random.default_rng(cols)
    X = rng.normal(size=(777, cols)) * rng.choice([0.01, 1.0, 30.0], size=(777, 1))
    X[::7, : cols // 2] = X[::7, :1]  # ties
    Y = _pdt.pdt_project_simplex(gpu(X, dev)).cpu().numpy()
    ref = simplex.project_rows(X)
    assert np.max(np.abs(Y - ref)) <= 1e-14 * max(1.0, np.max(np.abs(X)))
    assert np.all(Y >= 0)
    Yf = _pdt.pdt_project_simplex(gpu(X, dev, torch.float32)).cpu().numpy()
    assert np.max(np.abs(Yf - ref)) <= 2e-6 * max(1.0, np.max(np.abs(X)))


def test_projection_bruteforce_and_inplace(dev):
    rng = np.random.default_rng(3)
    X = rng.normal(size=(64, 7))
    T = gpu(X, dev)
    _pdt.pdt_project_simplex(T, T)  # in place
    for r in range(64):
        assert np.max(np.abs(T[r].cpu().numpy() - simplex.project_simplex_bruteforce(X[r]))) < 1e-14


def test_projection_empty(dev):
    T = torch.zeros((0, 5), dtype=torch.float64, device=dev)
    _pdt.pdt_project_simplex(T, T)


# ---- setup: bands, tail mass, Lipschitz constant -----------------------------------------

@pytest.mark.parametrize("which", ["c1", "c2", "small"])
def test_bands_and_lipschitz(dev, which):
    inst = {"c1": synth.c1_small, "c2": synth.c2_medium, "small": small_instance}[which]()
    pb = _pdt.Problem.from_instance(inst)
    b = pb.bands()
    lo, hi = poisson.bands(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    mism = np.nonzero((lo != b["lo"]) | (hi != b["hi"]))[0]
    # an edge may differ only where the entry sits on the threshold to rounding
    for d in mism:
        for e_o, e_g in ((lo[d], b["lo"][d]), (hi[d], b["hi"][d])):
            if e_o != e_g:
                assert abs(int(e_o) - int(e_g)) == 1
                m = max(e_o, e_g) if e_g > e_o else min(e_o, e_g)
                v = poisson.row_values(float(inst.mu[d]), int(m), int(m), inst.M, inst.tail_mode)[0]
                assert abs(v - inst.threshold) <= 1e-12 * inst.threshold
    assert len(mism) <= max(2, len(lo) // 1000)
    if inst.tail_mode == synth.LUMP:
        ref = np.array([poisson.upper_tail(float(m_), inst.M - 1) for m_ in inst.mu])
        # relative 1e-12 wherever the tail is representable at all (below 1e-30 it lies
        # far under the band threshold and either side may flush it to zero)
        assert np.all(np.abs(b["tail"] - ref) <= 1e-12 * ref + 1e-30)
    F, _, _ = oracle_F(inst)
    L = fista.lipschitz(F, inst.gamma, inst.M)
    assert b["lipschitz"] == pytest.approx(L, rel=1e-10)


# ---- objective and gradient ---------------------------------------------------------------

@pytest.mark.parametrize("which", ["c1", "c2", "small", "small_trunc", "ragged"])
def test_objective_and_gradient(dev, which):
    inst = {
        "c1": synth.c1_small,
        "c2": synth.c2_medium,
        "small": small_instance,
        "small_trunc": lambda: small_instance(tail=synth.TRUNCATE, mu_max=150.0, tau=0.0),
        "ragged": lambda: small_instance(M=37, B=4, D=23, mu_max=30.0),
    }[which]()
    F, _, _ = oracle_F(inst)
    rng = np.random.default_rng(11)
    pb = _pdt.Problem.from_instance(inst)
    for trial in range(3):
        Pi = simplex.project_rows(rng.normal(size=(inst.M, inst.N)) * [0.01, 1.0, 5.0][trial])
        G = torch.empty((inst.M, inst.N), dtype=torch.float64, device=dev)
        f = pb.objective(gpu(Pi, dev), G)
        fr = objective.objective(F, inst.P, Pi, inst.gamma)
        Gr = objective.gradient(F, inst.P, Pi, inst.gamma)
        assert f == pytest.approx(fr, rel=1e-12)
        assert np.max(np.abs(G.cpu().numpy() - Gr)) <= 1e-12 * np.max(np.abs(Gr))
        k = pb.kkt(gpu(Pi, dev))
        assert k == pytest.approx(certify.kkt_residual(F, inst.P, Pi, inst.gamma), rel=1e-9)


# ---- solver trajectory parity -----------------------------------------------------------

def run_both(inst, iters, precision=_pdt.PDT_FP64, dev=None):
    F, _, _ = oracle_F(inst)
    L = fista.lipschitz(F, inst.gamma, inst.M)
    ref = fista.fista_r(F, inst.P, inst.gamma, L, iters, exact_sums=False)
    pb = _pdt.Problem.from_instance(inst)
    Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
    hist = torch.zeros(max(iters, 1), dtype=torch.float64, device=dev)
    info = pb.solve(Pi, precision=precision, max_iters=iters, step_L=L, history=hist)
    return ref, Pi.cpu().numpy(), info, hist.cpu().numpy()[:iters], F


def test_trajectory_c1_fp64_2000(dev):
    inst = synth.c1_small()
    ref, Pi, info, hist, F = run_both(inst, 2000, dev=dev)
    assert info["iters"] == 2000
    assert abs(info["objective"] - ref.f) <= 1e-9 * ref.f
    assert np.max(np.abs(Pi - ref.X)) <= 1e-6
    assert np.all(np.diff(hist) <= 0)  # accepted objective never increases
    assert np.all(Pi >= 0) and np.max(np.abs(Pi.sum(1) - 1)) < 1e-14
    # every iterate's objective tracks the oracle's
    assert np.max(np.abs(hist - ref.history) / ref.history) < 1e-9


@pytest.mark.parametrize("which,iters", [("small", 400), ("ragged", 600), ("small_trunc", 300)])
def test_trajectory_fp64(dev, which, iters):
    inst = {
        "small": small_instance,
        "ragged": lambda: small_instance(M=37, B=4, D=23, mu_max=30.0),
        "small_trunc": lambda: small_instance(tail=synth.TRUNCATE, mu_max=150.0, tau=0.0),
    }[which]()
    ref, Pi, info, hist, F = run_both(inst, iters, dev=dev)
    assert abs(info["objective"] - ref.f) <= 1e-9 * ref.f
    assert np.max(np.abs(Pi - ref.X)) <= 1e-6


def test_trajectory_c2_fp64_short(dev):
    inst = synth.c2_medium()
    ref, Pi, info, hist, F = run_both(inst, 15, dev=dev)
    assert abs(info["objective"] - ref.f) <= 1e-9 * ref.f
    assert np.max(np.abs(Pi - ref.X)) <= 1e-6


def test_fp32_path_c1(dev):
    inst = synth.c1_small()
    ref, Pi, info, hist, F = run_both(inst, 2000, precision=_pdt.PDT_FP32, dev=dev)
    assert abs(info["objective"] - ref.f) <= 1e-4 * ref.f
    # Without FP64 refinement the FP32 iterate is only as good as conditioning allows:
    # kappa(2 F^T F + 2 gamma L) ~ 1.2e5 times FP32 rounding ~ 6e-8 gives ~1e-2
    assert np.max(np.abs(Pi - ref.X)) <= 5e-2
    assert np.all(Pi >= 0) and np.max(np.abs(Pi.sum(1) - 1)) < 1e-5


# ---- degenerate cases ----------------------------------------------------------------------

def test_single_outcome(dev):
    mu = np.linspace(0, 10, 12)
    P = np.ones((12, 1))
    pb = _pdt.Problem(mu, P, 16, 0.1, 0.0, _pdt.PDT_TAIL_TRUNCATE)
    Pi = torch.zeros((16, 1), dtype=torch.float64, device=dev)
    pb.solve(Pi, max_iters=10)
    assert torch.all(Pi == 1.0)


def test_vacuum_probe(dev):
    # one probe with mu = 0 sees only m = 0; with gamma > 0 every row tends to P_0
    M = 12
    P0 = np.array([[0.1, 0.2, 0.3, 0.4]])
    F = poisson.dense_F(np.array([0.0]), M, 0.0, poisson.TRUNCATE)
    L = fista.lipschitz(F, 1.0, M)
    pb = _pdt.Problem(np.array([0.0]), P0, M, 1.0, 0.0, _pdt.PDT_TAIL_TRUNCATE)
    Pi = torch.zeros((M, 4), dtype=torch.float64, device=dev)
    pb.solve(Pi, max_iters=5000, step_L=L)
    assert np.max(np.abs(Pi.cpu().numpy() - P0)) < 1e-8


def test_single_photon_number(dev):
    # M = 1: one row, lumped column holds all the mass; the solution is P_S(weighted mean of P)
    mu = np.array([0.0, 1.0, 3.0])
    P = simplex.project_rows(np.random.default_rng(2).random((3, 5)))
    inst_F = poisson.dense_F(mu, 1, 0.0, poisson.LUMP)
    assert np.allclose(inst_F, 1.0)
    pb = _pdt.Problem(mu, P, 1, 0.0, 1e-16, _pdt.PDT_TAIL_LUMP)
    Pi = torch.zeros((1, 5), dtype=torch.float64, device=dev)
    pb.solve(Pi, max_iters=500)
    ref = simplex.project_simplex(P.mean(0))
    assert np.max(np.abs(Pi.cpu().numpy()[0] - ref)) < 1e-12


def test_user_start_is_projected(dev):
    inst = small_instance(M=40, B=6, D=50, mu_max=45.0)
    pb = _pdt.Problem.from_instance(inst)
    X0 = np.random.default_rng(4).normal(size=(inst.M, inst.N))
    Pi = gpu(X0, dev)
    info = pb.solve(Pi, init=_pdt.PDT_INIT_USER, max_iters=0)
    assert info["iters"] == 0
    assert np.max(np.abs(Pi.cpu().numpy() - simplex.project_rows(X0))) < 1e-14


def test_tolerance_stop_and_not_converged(dev):
    inst = synth.c1_small()
    F, _, _ = oracle_F(inst)
    pb = _pdt.Problem.from_instance(inst)
    Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
    fstar = 0.0030297518638230363  # certified optimum of this instance (tests/golden/c1_oracle.json)
    info = pb.solve(Pi, max_iters=100000, rel_obj_tol=1e-6, f_star=fstar)
    assert info["status"] == _pdt.PDT_OK and info["converged"] == 1
    assert info["iters"] < 100000
    assert (info["objective"] - fstar) <= 1e-6 * fstar
    info2 = pb.solve(Pi, max_iters=10, rel_obj_tol=1e-12, f_star=fstar)
    assert info2["status"] == _pdt.PDT_ERR_NOT_CONVERGED and info2["iters"] == 10


# ---- mixed precision: FP32 products on FP64 iterates, then FP64 refinement ---------------

def _golden_c1():
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "c1_oracle.json")) as fh:
        return json.load(fh)


def test_mixed_reaches_the_certified_optimum_c1(dev):
    inst = synth.c1_small()
    gold = _golden_c1()
    fstar, Xstar = gold["f_star"], np.array(gold["Pi_star"])
    pb = _pdt.Problem.from_instance(inst)
    Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
    # An objective-monotone method stops moving along the flattest direction of this
    # ill-conditioned problem once the decrease, lambda_min * dX^2 ~ 3.4e-5 * dX^2, drops
    # below the FP64 rounding of f (~1e-15 * f): dX ~ 1e-6.  The oracle's own iteration
    # stalls there too (1.07e-6 after 20000 iterations), so the optimum bound is 2e-6.
    info = pb.solve(Pi, precision=_pdt.PDT_MIXED, max_iters=60000)
    assert info["status"] == _pdt.PDT_OK and info["iters"] == 60000
    X = Pi.cpu().numpy()
    assert abs(info["objective"] - fstar) <= 1e-12 * fstar
    assert np.max(np.abs(X - Xstar)) <= 2e-6
    assert np.all(X >= 0) and np.max(np.abs(X.sum(1) - 1)) < 1e-14


def test_mixed_early_iterates_track_fp64(dev):
    # before the refinement takes over, FP32 products keep the iterate within 1e-4
    inst = small_instance()
    F, _, _ = oracle_F(inst)
    L = fista.lipschitz(F, inst.gamma, inst.M)
    ref = fista.fista_r(F, inst.P, inst.gamma, L, 256, exact_sums=False)
    pb = _pdt.Problem.from_instance(inst)
    Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
    info = pb.solve(Pi, precision=_pdt.PDT_MIXED, max_iters=256, step_L=L)
    assert info["iters"] == 256
    assert abs(info["objective"] - ref.f) <= 1e-4 * ref.f
    assert np.max(np.abs(Pi.cpu().numpy() - ref.X)) <= 1e-4


def test_mixed_c2_tolerance(dev):
    # the mixed solve stops at the same relative objective as the FP64 one
    inst = synth.c2_medium()
    pb = _pdt.Problem.from_instance(inst)
    Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
    ref = pb.solve(Pi, max_iters=60000)
    fstar = ref["objective"]
    Pi.zero_()
    info = pb.solve(Pi, precision=_pdt.PDT_MIXED, max_iters=200000, rel_obj_tol=1e-6, f_star=fstar)
    assert info["converged"] == 1 and (info["objective"] - fstar) <= 1e-6 * fstar
    assert pb.kkt(Pi) < 1e-6
