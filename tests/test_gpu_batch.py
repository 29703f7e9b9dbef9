"""Batched solve: many instances of uneven M, N and D in one launch per phase.

Each instance runs the same kernel bodies with the same fixed-order reductions as a
single-instance solve, so the batched results must equal the single solves bit for bit;
one instance is also checked against the oracle's trajectory."""
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


def family(count=7, m_range=(37, 400), bins=(3, 40)):
    out = []
    for i in range(count):
        rng = synth.rng_for(44, spawn=i)
        M = int(rng.integers(m_range[0], m_range[1] + 1))
        out.append(synth.random_detector(rng, M, bins=bins, name=f"batch_{i}"))
    return out


@pytest.mark.parametrize("precision", [_pdt.PDT_FP64, _pdt.PDT_FP32])
def test_batch_equals_single_solves(dev, precision):
    insts = family()
    assert len({i.N for i in insts}) > 2 and len({i.M for i in insts}) > 2
    bp = _pdt.BatchProblem(insts)
    Pis = [torch.zeros((i.M, i.N), dtype=torch.float64, device=dev) for i in insts]
    infos = bp.solve(Pis, precision=precision, max_iters=300)
    for inst, Pi, info in zip(insts, Pis, infos):
        pb = _pdt.Problem.from_instance(inst)
        X = torch.zeros_like(Pi)
        single = pb.solve(X, precision=precision, max_iters=300)
        assert info["iters"] == single["iters"] == 300
        assert torch.equal(Pi, X)
        assert info["objective"] == single["objective"]


@pytest.mark.parametrize("precision", [_pdt.PDT_FP64, _pdt.PDT_FP32])
def test_batch_with_narrow_tiles_equals_single_solves(dev, precision):
    # few probes with wide bands: every 16-row tile meets only a few probes, so the single
    # solve runs the narrow-only transposed product; the batch must reproduce it bit for bit
    wide = [synth.make_instance(f"narrow_{k}", M=1500 + 500 * k, B=20 + 5 * k, eta=0.8, dark=1e-4, D=30 + 10 * k,
                                mu_max=1300.0 + 400 * k, shots=1e6, gamma=1e-4, tail_mode=synth.LUMP,
                                threshold=1e-16, rng=synth.rng_for(61, spawn=k)) for k in range(2)]
    insts = wide + family(count=2)
    bp = _pdt.BatchProblem(insts)
    Pis = [torch.zeros((i.M, i.N), dtype=torch.float64, device=dev) for i in insts]
    infos = bp.solve(Pis, precision=precision, max_iters=300)
    for inst, Pi, info in zip(insts, Pis, infos):
        pb = _pdt.Problem.from_instance(inst)
        X = torch.zeros_like(Pi)
        single = pb.solve(X, precision=precision, max_iters=300)
        assert info["iters"] == single["iters"] == 300
        assert torch.equal(Pi, X), inst.name
        assert info["objective"] == single["objective"]
        pb.close()


def test_batch_matches_oracle_and_stops_per_instance(dev):
    insts = family(count=5)
    bp = _pdt.BatchProblem(insts)
    # per-instance targets: a long single solve of each
    fstar = []
    for inst in insts:
        pb = _pdt.Problem.from_instance(inst)
        X = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
        fstar.append(pb.solve(X, max_iters=20000)["objective"])
    Pis = [torch.zeros((i.M, i.N), dtype=torch.float64, device=dev) for i in insts]
    infos = bp.solve(Pis, max_iters=20000, rel_obj_tol=1e-6, f_star=fstar)
    iters = [i["iters"] for i in infos]
    assert all(i["converged"] == 1 for i in infos)
    assert len(set(iters)) > 1  # instances stop on their own
    for inst, info, fs in zip(insts, infos, fstar):
        assert info["objective"] - fs <= 1e-6 * fs
    # trajectory of instance 0 against the oracle, same step
    inst = insts[0]
    F, _, _ = poisson.build_F(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    L = fista.lipschitz(F, inst.gamma, inst.M)
    ref = fista.fista_r(F, inst.P, inst.gamma, L, 200, exact_sums=False)
    Pis = [torch.zeros((i.M, i.N), dtype=torch.float64, device=dev) for i in insts]
    infos = bp.solve(Pis, max_iters=200, step_L=L)
    assert abs(infos[0]["objective"] - ref.f) <= 1e-9 * ref.f
    assert np.max(np.abs(Pis[0].cpu().numpy() - ref.X)) <= 1e-6
