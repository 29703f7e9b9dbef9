"""Full-size parity on the paper-scale workload: the beam-splitter loop detector of the
paper's experiment in synthetic form (M = 1,210,581, N = 151, D = 1076 probes with
mu_d = d^2, band of 8.9e6 F entries).  Bands up to ~1.8e4 entries wide with only 68
probe tiles, and ~47k rows above the last probe's band that only the regulariser
reaches.  GPU against the row-at-a-time oracle at sampled rows and probes.

Tolerances as for the M=1e6 problem: band edges exact (or off by one on the
threshold); Hessian diagonal 1e-12 relative; gradient and Hessian-product rows 1e-10 of
their largest entry; one FP64 step 1e-9 absolute; one mixed step 1e-4.
"""
import os

import numpy as np
import pytest

from oracle import poisson, sampled, simplex
from paper_2404_02844_amd import _pdt, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PROBES = [0, 1, 2, 500, 1074, 1075]


@pytest.fixture(scope="module")
def loop():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pdt.lib()
    print("\n[loop] generating the paper-scale problem", flush=True)
    inst = synth.loop_paper_scale(workers=min(16, os.cpu_count() or 1))
    rows = [0, 1, 777, 250000, 1000000, 1163000, 1200000, inst.M - 1]
    print("[loop] setting up on the GPU", flush=True)
    pb = _pdt.Problem.from_instance(inst)
    ro = sampled.RowOracle(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    rng = np.random.default_rng(41)
    Pi = rng.random((inst.M, inst.N))
    Pi /= Pi.sum(axis=1, keepdims=True)
    print("[loop] oracle gradient rows", flush=True)
    G_rows = ro.gradient_rows(inst.P, Pi, inst.gamma, rows)
    yield inst, pb, ro, Pi, G_rows, rows
    pb.close()


def test_loop_bands_and_hessian_diag(loop):
    inst, pb, ro, _, _, rows = loop
    b = pb.bands()
    print(f"[loop] band entries {b['nnz']:.4e}, L = {b['lipschitz']:.4e}")
    assert 8.5e6 < b["nnz"] < 9.3e6
    for d in PROBES:
        lo, hi = ro.edges(d)
        for e_o, e_g in ((lo, int(b["lo"][d])), (hi, int(b["hi"][d]))):
            if e_o != e_g:
                assert abs(e_o - e_g) == 1, (d, e_o, e_g)
                v = float(poisson.pmf(max(e_o, e_g) if e_g > e_o else min(e_o, e_g), float(inst.mu[d]))[0])
                assert abs(v - inst.threshold) <= 1e-12 * inst.threshold, (d, v)
    assert int(b["hi"].max()) < inst.M - 1  # the top rows are reached by no probe
    h = ro.hessian_diag_rows(inst.gamma, rows)
    assert np.max(np.abs(pb.scaling()["hdiag"][rows] - h) / h) <= 1e-12


def test_loop_gradient_and_hessian_rows(loop):
    inst, pb, ro, Pi, G_rows, rows = loop
    G = torch.empty((inst.M, inst.N), dtype=torch.float64, device="cuda")
    pb.objective(torch.as_tensor(Pi, device="cuda"), G)
    assert np.max(np.abs(G[rows].cpu().numpy() - G_rows)) <= 1e-10 * np.max(np.abs(G_rows))
    # Hessian product = gradient of the same point against zero data
    HV = torch.empty_like(G)
    pb.hessian(torch.as_tensor(Pi, device="cuda"), HV)
    H_rows = ro.gradient_rows(np.zeros_like(inst.P), Pi, inst.gamma, rows)
    assert np.max(np.abs(HV[rows].cpu().numpy() - H_rows)) <= 1e-10 * np.max(np.abs(H_rows))


@pytest.mark.parametrize("precision,tol", [(_pdt.PDT_FP64, 1e-9), (_pdt.PDT_MIXED, 1e-4)])
def test_loop_one_scaled_step(loop, precision, tol):
    inst, pb, ro, Pi, G_rows, rows = loop
    Lw = pb.scaling()["lipschitz_scaled"]
    h = ro.hessian_diag_rows(inst.gamma, rows)
    X = torch.as_tensor(Pi, device="cuda").contiguous()
    info = pb.solve(X, init=_pdt.PDT_INIT_USER, precision=precision, max_iters=1, step_L=Lw,
                    scaling=_pdt.PDT_STEP_DIAG)
    assert info["iters"] == 1 and info["rejects"] == 0
    ref = simplex.project_rows(Pi[rows] - (1.0 / h / Lw)[:, None] * G_rows)
    got = X[rows].cpu().numpy()
    print(f"[loop] one step, precision {precision}: max |dPi| = {np.max(np.abs(got - ref)):.3e}")
    assert np.max(np.abs(got - ref)) <= tol
