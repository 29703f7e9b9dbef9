"""Degenerate problems through the Newton-CG, smoothing and Hessian entry points:
a single outcome (N = 1: every row is the vertex 1), a single photon number (M = 1),
a single probe (D = 1), and rows no probe reaches with gamma = 0.  The GPU must return
the oracle's iterate and decisions (4 CG iterations per step, as in the trajectory
tests) and stay feasible."""
import numpy as np
import pytest

from oracle import fista, newton, poisson, smoothing, simplex
from paper_2404_02844_amd import _pdt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pdt.lib()
    return torch.device("cuda:0")


def problem(M, N, D, gamma, seed=0, mu_max=20.0, tau=0.0, tail=_pdt.PDT_TAIL_TRUNCATE):
    rng = np.random.default_rng(seed)
    mu = np.linspace(0.0, mu_max, D)
    P = rng.random((D, N))
    P /= P.sum(axis=1, keepdims=True)
    return mu, P, M, gamma, tau, tail


CASES = {
    "one_outcome": problem(30, 1, 12, 1e-3),
    "one_photon_number": problem(1, 5, 7, 1e-3),
    "one_probe": problem(25, 4, 1, 1e-2, mu_max=3.0),
    "uncovered_rows_gamma0": problem(60, 3, 6, 0.0, mu_max=8.0, tau=1e-16),
}


@pytest.mark.parametrize("which", list(CASES))
def test_newton_edge_cases_follow_the_oracle(dev, which):
    mu, P, M, gamma, tau, tail = CASES[which]
    N = P.shape[1]
    F, _, _ = poisson.build_F(mu, M, tau, tail)
    ref = newton.two_stage(F, P, gamma, max_newton=5, eps_kkt=0.0, cg_max=4)
    pb = _pdt.Problem(mu, P, M, gamma, tau, tail)
    Pi = torch.empty((M, N), dtype=torch.float64, device=dev)
    r = pb.newton(Pi, max_newton=5, eps_kkt=0.0, cg_max=4)
    X = Pi.cpu().numpy()
    assert (r["stage1_iters"], r["stage2_iters"]) == (ref.stage1_iters, ref.stage2_iters)
    assert np.max(np.abs(X - ref.X)) <= 1e-9
    assert np.all(X >= 0) and np.max(np.abs(X.sum(axis=1) - 1)) <= 1e-13
    if N == 1:
        assert np.all(X == 1.0)
    # Hessian product against the oracle's
    V = np.random.default_rng(2).normal(size=(M, N))
    HV = torch.empty_like(Pi)
    pb.hessian(torch.as_tensor(V, device=dev), HV)
    href = fista.hessian_apply(F, gamma, V)
    assert np.max(np.abs(HV.cpu().numpy() - href)) <= 1e-12 * max(1e-300, np.max(np.abs(href)))
    pb.close()


@pytest.mark.parametrize("M,N,divisor,skip", [(1, 1, 1, 0), (2, 3, 1, 0), (5, 2, 1, 100), (9, 4, 1, 0)])
def test_smoothing_edge_cases(dev, M, N, divisor, skip):
    Pi = simplex.project_rows(np.random.default_rng(M).normal(size=(M, N)))
    out = _pdt.pdt_smooth_rows(torch.as_tensor(Pi, device=dev), divisor=divisor, skip=skip).cpu().numpy()
    assert np.max(np.abs(out - smoothing.smooth_rows(Pi, divisor, skip))) <= 1e-15


def test_invalid_smoothing_arguments(dev):
    Pi = torch.full((4, 2), 0.5, dtype=torch.float64, device=dev)
    for kw in (dict(divisor=0), dict(skip=-1)):
        with pytest.raises(_pdt.PdtError) as ei:
            _pdt.pdt_smooth_rows(Pi, **kw)
        assert ei.value.status == _pdt.PDT_ERR_INVALID_ARG
