"""Both workgroup shapes of the band kernels (4 or 8 waves splitting each tile's
contraction) against the FP64 oracle, and the batch reproducing single solves bit for
bit under a forced shape."""
import numpy as np
import pytest

from oracle import fista, poisson
from paper_2404_02844_amd import _pdt, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pdt.lib()
    return torch.device("cuda:0")


def instance(M=300, B=40, seed=3):
    rng = synth.rng_for(47, spawn=seed)
    return synth.random_detector(rng, M, bins=(B, B), name=f"tiles_{M}_{B}")


@pytest.mark.parametrize("ks_fx,ks_ftr", [(4, 4), (8, 8), (4, 8), (8, 4)])
@pytest.mark.parametrize("precision,tol_f,tol_x", [(_pdt.PDT_FP64, 1e-9, 1e-6), (_pdt.PDT_MIXED, 1e-4, 1e-4)])
def test_shapes_match_the_oracle(dev, ks_fx, ks_ftr, precision, tol_f, tol_x):
    inst = instance()
    F, _, _ = poisson.build_F(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    w = fista.row_weights(F, inst.gamma, inst.M)
    Lw = fista.lipschitz_scaled(F, inst.gamma, inst.M, w)
    ref = fista.fista_r(F, inst.P, inst.gamma, Lw, 300, exact_sums=False, row_w=w)
    pb = _pdt.Problem.from_instance(inst)
    pb.set_tiles(precision, ks_fx, ks_ftr)
    assert pb.tiles(precision) == (ks_fx, ks_ftr)
    Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
    info = pb.solve(Pi, precision=precision, max_iters=300, step_L=Lw, scaling=_pdt.PDT_STEP_DIAG)
    assert info["iters"] == 300
    assert abs(info["objective"] - ref.f) <= tol_f * ref.f
    assert np.max(np.abs(Pi.cpu().numpy() - ref.X)) <= tol_x


def test_fp32_shapes_agree(dev):
    inst = instance(M=700, B=100)
    pb = _pdt.Problem.from_instance(inst)
    out = []
    for ks in (4, 8):
        pb.set_tiles(_pdt.PDT_FP32, ks, ks)
        Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
        out.append((pb.solve(Pi, precision=_pdt.PDT_FP32, max_iters=200)["objective"], Pi.cpu().numpy()))
    assert abs(out[0][0] - out[1][0]) <= 1e-4 * out[0][0]
    assert np.max(np.abs(out[0][1] - out[1][1])) <= 1e-3


def test_bad_shapes_are_rejected(dev):
    pb = _pdt.Problem.from_instance(instance(M=40, B=4))
    for ks in (2, 16, -4):
        with pytest.raises(_pdt.PdtError):
            pb.set_tiles(_pdt.PDT_FP64, ks, 4)
    assert pb.tiles(_pdt.PDT_FP64) in ((4, 4), (8, 4), (4, 8), (8, 8))


@pytest.mark.parametrize("precision", [_pdt.PDT_FP64, _pdt.PDT_FP32])
def test_batch_with_forced_shape_equals_single_solves(dev, precision):
    insts = [instance(M=int(m), B=int(b), seed=i) for i, (m, b) in enumerate([(90, 8), (300, 40), (555, 100), (61, 20)])]
    bp = _pdt.BatchProblem(insts)
    for k in range(len(insts)):
        _pdt.pdt_problem_set_tiles(bp.handle, k, precision, 8, 8 if k % 2 else 4)
    Pis = [torch.zeros((i.M, i.N), dtype=torch.float64, device=dev) for i in insts]
    infos = bp.solve(Pis, precision=precision, max_iters=200, scaling=_pdt.PDT_STEP_DIAG)
    for k, (inst, Pi, info) in enumerate(zip(insts, Pis, infos)):
        pb = _pdt.Problem.from_instance(inst)
        pb.set_tiles(precision, 8, 8 if k % 2 else 4)
        X = torch.zeros_like(Pi)
        single = pb.solve(X, precision=precision, max_iters=200, scaling=_pdt.PDT_STEP_DIAG)
        assert torch.equal(Pi, X), k
        assert info["objective"] == single["objective"]
