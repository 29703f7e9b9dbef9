"""Split contractions of the two band products (several workgroups per 16-probe tile of
the forward product, or per 16-row tile of the transposed product, partial tiles summed
in a fixed order by the last of them) against the FP64 oracle and against the unsplit
launch, through the C ABI.

Forced splits on small problems exercise every launch mode that goes through the band
products: the momentum iteration (FP64, FP32, mixed with its delta products and
resyncs), plain evaluations, Newton-CG's Hessian products and objective evaluations.
Tolerances as in the unsplit tests (the split changes only the order of the sums):
trajectories 1e-9 relative f / 1e-6 max |dPi|; objective and gradient 1e-12; Newton
steps with 4 CG iterations 1e-9; a given split is deterministic bit for bit.
"""
import numpy as np
import pytest

from oracle import fista, newton, objective, poisson, simplex
from paper_2404_02844_amd import _pdt, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pdt.lib()
    return torch.device("cuda:0")


def small_instance(M=200, B=20, D=300, mu_max=220.0, gamma=1e-3, tail=synth.LUMP, tau=1e-16, seed=7):
    return synth.make_instance(f"small_m{M}_b{B}_d{D}", M=M, B=B, eta=0.8, dark=1e-4, D=D, mu_max=mu_max,
                               shots=1e6, gamma=gamma, tail_mode=tail, threshold=tau, rng=synth.rng_for(90 + seed))


INSTANCES = {
    "c1": synth.c1_small,
    "small": small_instance,
    # few probes with wide bands: long photon-number ranges per probe tile
    "wideband": lambda: small_instance(M=3000, B=30, D=40, mu_max=2700.0, gamma=1e-4),
    "ragged": lambda: small_instance(M=37, B=4, D=23, mu_max=30.0),
    # many probes per row: ~30 64-probe chunks per row tile of the transposed product
    "denseband": lambda: small_instance(M=300, B=24, D=2000, mu_max=330.0, gamma=1e-4),
}
_cache = {}


def setup(which):
    if which not in _cache:
        inst = INSTANCES[which]()
        F, _, _ = poisson.build_F(inst.mu, inst.M, inst.threshold, inst.tail_mode)
        _cache[which] = (inst, F, fista.lipschitz(F, inst.gamma, inst.M))
    return _cache[which]


def set_split(pb, kind, split):
    getattr(pb, f"set_{kind}_split")(split)
    return getattr(pb, f"{kind}_split")()


@pytest.mark.parametrize("kind", ["fx", "ftr"])
@pytest.mark.parametrize("split", [2, 3, 8, 16])
@pytest.mark.parametrize("which", list(INSTANCES))
def test_split_trajectory_matches_oracle(dev, which, split, kind):
    inst, F, L = setup(which)
    print(f"[split] {kind} {which} split {split}", flush=True)
    pb = _pdt.Problem.from_instance(inst)
    assert set_split(pb, kind, split) == split
    iters = 200
    ref = fista.fista_r(F, inst.P, inst.gamma, L, iters)
    Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
    info = pb.solve(Pi, max_iters=iters, step_L=L)
    assert abs(info["objective"] - ref.f) <= 1e-9 * ref.f
    assert np.max(np.abs(Pi.cpu().numpy() - ref.X)) <= 1e-6
    # objective and gradient at a random feasible point
    X = simplex.project_rows(np.random.default_rng(split).normal(size=(inst.M, inst.N)))
    G = torch.empty_like(Pi)
    f = pb.objective(torch.as_tensor(X, device=dev), G)
    assert f == pytest.approx(objective.objective(F, inst.P, X, inst.gamma), rel=1e-12)
    gref = objective.gradient(F, inst.P, X, inst.gamma)
    assert np.max(np.abs(G.cpu().numpy() - gref)) <= 1e-12 * np.max(np.abs(gref))
    # Newton-CG: Hessian products and line-search evaluations go through the split launch
    nref = newton.two_stage(F, inst.P, inst.gamma, max_newton=2, eps_kkt=0.0, cg_max=4)
    r = pb.newton(Pi, max_newton=2, eps_kkt=0.0, cg_max=4)
    assert r["stage1_iters"] == nref.stage1_iters
    assert np.max(np.abs(Pi.cpu().numpy() - nref.X)) <= 1e-9
    pb.close()


@pytest.mark.parametrize("kind,which", [("fx", "wideband"), ("fx", "small"), ("ftr", "denseband"),
                                        ("ftr", "small")])
def test_split_is_deterministic_and_close_to_unsplit(dev, which, kind):
    inst, F, L = setup(which)
    pb = _pdt.Problem.from_instance(inst)
    out = {}
    for split in (1, 4, 4):
        set_split(pb, kind, split)
        Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
        info = pb.solve(Pi, max_iters=300, scaling=_pdt.PDT_STEP_DIAG)
        out.setdefault(split, []).append((info["objective"], Pi.cpu().numpy()))
    (f1, X1), = out[1]
    (fa, Xa), (fb, Xb) = out[4]
    assert fa == fb and np.array_equal(Xa, Xb)  # bit for bit
    assert abs(fa - f1) <= 1e-12 * f1 and np.max(np.abs(Xa - X1)) <= 1e-9
    set_split(pb, kind, 0)
    pb.close()


@pytest.mark.parametrize("kind,which", [("fx", "wideband"), ("ftr", "denseband")])
@pytest.mark.parametrize("precision,tol", [(_pdt.PDT_MIXED, 1e-4), (_pdt.PDT_FP32, 1e-3)])
def test_split_reduced_precision_paths(dev, precision, tol, kind, which):
    inst, F, L = setup(which)
    pb = _pdt.Problem.from_instance(inst)
    res = {}
    for split in (1, 5):
        set_split(pb, kind, split)
        Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
        info = pb.solve(Pi, precision=precision, max_iters=400, scaling=_pdt.PDT_STEP_DIAG)
        res[split] = info["objective"]
    Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
    f64 = pb.solve(Pi, precision=_pdt.PDT_FP64, max_iters=400, scaling=_pdt.PDT_STEP_DIAG)["objective"]
    assert abs(res[5] - f64) <= tol * f64 and abs(res[1] - f64) <= tol * f64
    pb.close()


def test_automatic_choice(dev):
    # up to 16 workgroups per tile when there are fewer than 256 probe tiles (about 768 in
    # all), at least 32 64-entry chunks per workgroup: 3 tiles of up to ~250 chunks here
    inst = small_instance(M=40000, B=30, D=40, mu_max=36000.0, gamma=1e-4)
    lo, hi = poisson.bands(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    tiles = (inst.D + 15) // 16
    maxch = max((hi[t:t + 16].max() - lo[t:t + 16].min()) // 64 + 1 for t in range(0, inst.D, 16))
    expected = max(1, min(16, (768 + tiles - 1) // tiles, maxch // 32))
    pb = _pdt.Problem.from_instance(inst)
    assert expected > 1 and pb.fx_split() == expected
    X = simplex.project_rows(np.random.default_rng(3).normal(size=(inst.M, inst.N)))
    Xg = torch.as_tensor(X, device=dev)
    f_auto = pb.objective(Xg)
    pb.set_fx_split(1)
    assert pb.objective(Xg) == pytest.approx(f_auto, rel=1e-13)
    pb.close()
    pb = _pdt.Problem.from_instance(synth.c1_small())
    assert pb.fx_split() == 1  # one chunk per tile: nothing to split
    pb.close()
