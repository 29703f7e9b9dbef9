"""Full-size parity on the M=1e6, N=100, D=1e5 problem (99-bin detector with crosstalk,
a band of ~9.3e8 F entries that is never stored): the GPU against the row-at-a-time
oracle at sampled rows and probes, and closed forms that hold at any size.

Tolerances: band edges exact (or off by one where the entry sits on the threshold);
Hessian diagonal 1e-12 relative; objective at Pi = 1/N 1e-10 relative to the closed
form; gradient rows 1e-10 of their largest entry; one FP64 step 1e-9 absolute on the
sampled rows of Pi; one mixed-precision step 1e-4 (the mixed-path bound).
"""
import math
import os

import numpy as np
import pytest

from oracle import poisson, sampled, simplex
from paper_2404_02844_amd import _pdt, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROWS = [0, 1, 12345, 500000, 777777]
PROBES = [0, 1, 5000, 45454, 90000, 99999]


@pytest.fixture(scope="module")
def c3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pdt.lib()
    print("\n[c3] generating the M=1e6 problem", flush=True)
    inst = synth.c3_mega(workers=min(16, os.cpu_count() or 1))
    print("[c3] setting up on the GPU", flush=True)
    pb = _pdt.Problem.from_instance(inst)
    ro = sampled.RowOracle(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    rng = np.random.default_rng(31)
    Pi = rng.random((inst.M, inst.N))
    Pi /= Pi.sum(axis=1, keepdims=True)
    print("[c3] oracle gradient rows", flush=True)
    G_rows = ro.gradient_rows(inst.P, Pi, inst.gamma, ROWS)
    return inst, pb, ro, Pi, G_rows


def test_c3_bands_and_hessian_diag(c3):
    inst, pb, ro, _, _ = c3
    b = pb.bands()
    print(f"[c3] band entries {b['nnz']:.4e}, L = {b['lipschitz']:.4e}")
    assert 9.0e8 < b["nnz"] < 9.6e8
    for d in PROBES:
        lo, hi = ro.edges(d)
        for e_o, e_g in ((lo, int(b["lo"][d])), (hi, int(b["hi"][d]))):
            if e_o != e_g:
                # an edge may move by one only where the entry sits on the threshold
                assert abs(e_o - e_g) == 1, (d, e_o, e_g)
                v = float(poisson.pmf(max(e_o, e_g) if e_g > e_o else min(e_o, e_g), float(inst.mu[d]))[0])
                assert abs(v - inst.threshold) <= 1e-12 * inst.threshold, (d, v)
    sc = pb.scaling()
    h = ro.hessian_diag_rows(inst.gamma, ROWS)
    assert np.max(np.abs(sc["hdiag"][ROWS] - h) / h) <= 1e-12
    assert math.isfinite(sc["lipschitz_scaled"]) and sc["lipschitz_scaled"] > 0


def test_c3_objective_at_uniform_start(c3):
    # F 1 = 1 (rows of the lumped F sum to one), so F (1/N) = 1/N and f = ||1/N - P||^2
    inst, pb, _, _, _ = c3
    Pi = torch.full((inst.M, inst.N), 1.0 / inst.N, dtype=torch.float64, device="cuda")
    f = pb.objective(Pi)
    ref = math.fsum(((1.0 / inst.N - inst.P) ** 2).ravel())
    assert f == pytest.approx(ref, rel=1e-10)


def test_c3_gradient_rows(c3):
    inst, pb, _, Pi, G_rows = c3
    G = torch.empty((inst.M, inst.N), dtype=torch.float64, device="cuda")
    pb.objective(torch.as_tensor(Pi, device="cuda"), G)
    got = G[ROWS].cpu().numpy()
    scale = np.max(np.abs(G_rows))
    assert np.max(np.abs(got - G_rows)) <= 1e-10 * scale


def test_c3_hessian_rows(c3):
    # Newton-CG's Hessian product at full size: the gradient of the same point against
    # zero data, from the row-at-a-time oracle
    inst, pb, ro, Pi, _ = c3
    HV = torch.empty((inst.M, inst.N), dtype=torch.float64, device="cuda")
    pb.hessian(torch.as_tensor(Pi, device="cuda"), HV)
    ref = ro.gradient_rows(np.zeros_like(inst.P), Pi, inst.gamma, ROWS)
    assert np.max(np.abs(HV[ROWS].cpu().numpy() - ref)) <= 1e-10 * np.max(np.abs(ref))


@pytest.mark.parametrize("precision,tol", [(_pdt.PDT_FP64, 1e-9), (_pdt.PDT_MIXED, 1e-4)])
def test_c3_one_scaled_step(c3, precision, tol):
    # from Pi (a feasible start) the first step has no momentum:
    # X_1[m] = P_S(Pi[m] - (w_m / L_w) grad_m), with w_m = 1 / h_m
    inst, pb, ro, Pi, G_rows = c3
    Lw = pb.scaling()["lipschitz_scaled"]
    h = ro.hessian_diag_rows(inst.gamma, ROWS)
    X = torch.as_tensor(Pi, device="cuda").contiguous()
    info = pb.solve(X, init=_pdt.PDT_INIT_USER, precision=precision, max_iters=1, step_L=Lw,
                    scaling=_pdt.PDT_STEP_DIAG)
    assert info["iters"] == 1 and info["rejects"] == 0
    ref = simplex.project_rows(Pi[ROWS] - (1.0 / h / Lw)[:, None] * G_rows)
    got = X[ROWS].cpu().numpy()
    print(f"[c3] one step, precision {precision}: max |dPi| = {np.max(np.abs(got - ref)):.3e}")
    assert np.max(np.abs(got - ref)) <= tol


def test_c3_iterations_descend_and_mixed_tracks_fp64(c3):
    inst, pb, _, _, _ = c3
    K = 64
    out = {}
    for precision in (_pdt.PDT_FP64, _pdt.PDT_MIXED):
        X = torch.zeros((inst.M, inst.N), dtype=torch.float64, device="cuda")
        hist = torch.zeros(K, dtype=torch.float64, device="cuda")
        info = pb.solve(X, precision=precision, max_iters=K, history=hist, scaling=_pdt.PDT_STEP_DIAG)
        h = hist.cpu().numpy()
        assert info["iters"] == K and np.all(np.diff(h) <= 0)
        rows = X[ROWS].cpu().numpy()
        assert np.all(rows >= 0) and np.max(np.abs(rows.sum(axis=1) - 1)) <= 1e-13
        out[precision] = (info["objective"], rows)
        print(f"[c3] {K} iterations, precision {precision}: f = {info['objective']:.6e}, "
              f"{info['seconds']:.2f} s")
    f64, r64 = out[_pdt.PDT_FP64]
    fmx, rmx = out[_pdt.PDT_MIXED]
    assert abs(fmx - f64) <= 1e-4 * f64
    assert np.max(np.abs(rmx - r64)) <= 1e-4
