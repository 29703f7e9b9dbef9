"""Two-stage two-metric projected Newton method (App. B, Algorithms 1-3) on the GPU vs
the FP64 oracle, through the C ABI.

CG in finite precision amplifies rounding: on the M=64 problem the oracle's own stage-1
direction moves by 3e-14 (10 iterations), 4e-7 (20) and 7e-4 (50) relative when its
Hessian products are perturbed by 1e-15 relative, while the CG model value
q(p) = p'Dp/2 + g'p it minimises moves by 5e-9 at 50 iterations.  Hence:
  * Hessian products: 1e-12 of max |HV| (one band product each way);
  * directions with at most 10 CG iterations: the same iteration count, max |dDir| <=
    1e-9 max |Dir|; slope 1e-9 relative in stage 2 (exact formula), 1e-6 in stage 1 (a
    difference quotient at alpha = 1e-9, whose rounding is ~1e-7 of X per entry);
  * directions with 50 CG iterations: model value within 1e-6 relative of the
    oracle's and a relative residual within 2x of the oracle's, both measured by the
    oracle's own operator;
  * whole solves with 4 CG iterations per step (where the oracle perturbed by 1e-15
    moves its 6-step iterate by <= 6e-12, against 4e-8 with 10 iterations and a
    different trajectory altogether on the gamma = 0 problem): identical decisions
    (stage counts, CG iterations), iterates within 1e-9, objective history 1e-10;
  * whole solves with 50: final objective within 1e-8 of the certified optimum of the
    M=64 problem, like the oracle's.
"""
import json
import os

import numpy as np
import pytest

from oracle import certify, fista, newton, objective, poisson, sampled, simplex
from paper_2404_02844_amd import _pdt, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


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
    "small_trunc": lambda: small_instance(tail=synth.TRUNCATE, mu_max=150.0, tau=0.0),
    "ragged": lambda: small_instance(M=37, B=4, D=23, mu_max=30.0),
    # 130 outcomes: three 64-column slices per row in the row kernels, 9 column tiles
    "wide": lambda: small_instance(M=150, B=129, D=90, mu_max=140.0, gamma=1e-2),
    # gamma = 0 with rows beyond every probe's band: zero Hessian diagonal entries
    "gamma0": lambda: small_instance(M=120, B=6, D=40, mu_max=30.0, gamma=0.0, tail=synth.TRUNCATE),
}

_cache = {}


def setup(which):
    if which not in _cache:
        inst = INSTANCES[which]()
        F, _, _ = poisson.build_F(inst.mu, inst.M, inst.threshold, inst.tail_mode)
        _cache[which] = (inst, F)
    inst, F = _cache[which]
    return inst, F, _pdt.Problem.from_instance(inst)


def random_point(inst, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return simplex.project_rows(rng.normal(size=(inst.M, inst.N)) * scale)


def gpu(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


@pytest.mark.parametrize("which", list(INSTANCES))
def test_hessian_apply_matches_oracle(dev, which):
    inst, F, pb = setup(which)
    print(f"[newton] hessian {which} M={inst.M} N={inst.N} D={inst.D}", flush=True)
    V = np.random.default_rng(3).normal(size=(inst.M, inst.N))
    HV = torch.empty((inst.M, inst.N), dtype=torch.float64, device=dev)
    pb.hessian(gpu(V, dev), HV)
    ref = fista.hessian_apply(F, inst.gamma, V)
    assert np.max(np.abs(HV.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))
    pb.close()


def oracle_direction(inst, F, X, stage, cg_max):
    g = objective.gradient(F, inst.P, X, inst.gamma)
    h = fista.hessian_diag(F, inst.gamma, inst.M)
    if stage == 1:
        eps = newton.binding_eps_stage1(X, g)
        D, it, bind = newton.stage1_direction(F, inst.gamma, X, g, h, eps, 1e-4, cg_max)
        slope = newton.stage1_slope(X, D, g)
        free, mi, gr = ~bind, None, g
        hd = np.where(h > 0, h, 1.0)[:, None]

        def op(v):
            return (np.where(free, fista.hessian_apply(F, inst.gamma, np.where(free, v, 0.0)), 0.0)
                    + np.where(bind, hd * v, 0.0))
    else:
        eps = newton.binding_eps_stage2(X, g, newton.reduce_max(X))
        D, it, mi, bind = newton.stage2_direction(F, inst.gamma, X, g, h, eps, 1e-4, cg_max)
        slope = newton.stage2_slope(X, D, g, mi)
        var = np.ones(X.shape, dtype=bool)
        var[np.arange(inst.M), mi] = False
        free = var & ~bind
        gr = np.where(var, newton.contract(g, mi), 0.0)
        hd = np.where(h > 0, 2.0 * h, 1.0)[:, None]

        def op(v):
            w = newton.contract(fista.hessian_apply(F, inst.gamma, newton.expand(np.where(free, v, 0.0), mi)), mi)
            return np.where(free, w, 0.0) + np.where(bind, hd * v, 0.0)
    return dict(D=D, it=it, slope=slope, eps=eps, mi=mi, op=op, g=gr)


def gpu_direction(pb, inst, X, stage, eps, cg_max, dev):
    Dg = torch.empty((inst.M, inst.N), dtype=torch.float64, device=dev)
    mi = torch.full((inst.M,), -1, dtype=torch.int32, device=dev)
    r = pb.newton_direction(stage, gpu(X, dev), eps, 1e-4, cg_max, Dg, mi)
    return Dg.cpu().numpy(), mi.cpu().numpy(), r


@pytest.mark.parametrize("stage", [1, 2])
@pytest.mark.parametrize("which", list(INSTANCES))
def test_direction_matches_oracle(dev, which, stage):
    inst, F, pb = setup(which)
    print(f"[newton] direction {which} stage {stage}", flush=True)
    X = random_point(inst, 11 + stage)
    ref = oracle_direction(inst, F, X, stage, 10)
    D, mi, r = gpu_direction(pb, inst, X, stage, ref["eps"], 10, dev)
    assert r["cg_iters"] == ref["it"]
    assert np.max(np.abs(D - ref["D"])) <= 1e-9 * np.max(np.abs(ref["D"]))
    assert r["slope"] == pytest.approx(ref["slope"], rel=1e-6 if stage == 1 else 1e-9)
    if stage == 2:
        assert np.array_equal(mi, ref["mi"])
        assert np.all(D[np.arange(inst.M), ref["mi"]] == 0.0)
    pb.close()


@pytest.mark.parametrize("cg_max", [1, 3, 4, 5, 7, 8, 9])
def test_direction_across_graph_boundaries(dev, cg_max):
    """CG iterations go out four per recorded graph and the remainder one by one; every
    split of cg_max gives the oracle's iteration count and direction."""
    inst, F, pb = setup("small")
    print(f"[newton] direction small stage 1 cg_max={cg_max}", flush=True)
    X = random_point(inst, 31)
    ref = oracle_direction(inst, F, X, 1, cg_max)
    D, _, r = gpu_direction(pb, inst, X, 1, ref["eps"], cg_max, dev)
    assert r["cg_iters"] == ref["it"]
    assert np.max(np.abs(D - ref["D"])) <= 1e-9 * np.max(np.abs(ref["D"]))
    pb.close()


def test_hessian_after_a_finished_solve(dev):
    """A conjugate-gradient solve ends with its stop flag set, which its own Hessian
    products skip on; a later plain Hessian product must still be computed."""
    inst, F, pb = setup("small")
    print("[newton] hessian after direction", flush=True)
    X = random_point(inst, 41)
    ref = oracle_direction(inst, F, X, 2, 6)
    gpu_direction(pb, inst, X, 2, ref["eps"], 6, dev)
    V = np.random.default_rng(5).normal(size=(inst.M, inst.N))
    HV = torch.empty((inst.M, inst.N), dtype=torch.float64, device=dev)
    pb.hessian(gpu(V, dev), HV)
    ref_hv = fista.hessian_apply(F, inst.gamma, V)
    assert np.max(np.abs(HV.cpu().numpy() - ref_hv)) <= 1e-12 * np.max(np.abs(ref_hv))
    pb.close()


@pytest.mark.parametrize("stage", [1, 2])
@pytest.mark.parametrize("which", ["c1", "small", "wide", "gamma0"])
def test_full_cg_direction_properties(dev, which, stage):
    inst, F, pb = setup(which)
    print(f"[newton] 50-iteration direction {which} stage {stage}", flush=True)
    X = random_point(inst, 21 + stage)
    ref = oracle_direction(inst, F, X, stage, 50)
    D, _, r = gpu_direction(pb, inst, X, stage, ref["eps"], 50, dev)
    op, g = ref["op"], ref["g"]

    def q(d):
        return 0.5 * np.sum(d * op(d)) + np.sum(g * d)

    def res(d):
        return np.linalg.norm(op(d) + g) / np.linalg.norm(g)

    assert r["cg_iters"] == ref["it"] or min(r["cg_iters"], ref["it"]) >= 45
    assert q(D) == pytest.approx(q(ref["D"]), rel=1e-6)
    assert res(D) <= 2.0 * res(ref["D"]) + 1e-12
    assert r["slope"] < 0
    pb.close()


@pytest.mark.parametrize("steps", [1, 2, 3, 6])
@pytest.mark.parametrize("which", ["c1", "small", "wide", "ragged", "gamma0"])
def test_first_steps_follow_the_oracle(dev, which, steps):
    inst, F, pb = setup(which)
    print(f"[newton] first {steps} steps {which}", flush=True)
    ref = newton.two_stage(F, inst.P, inst.gamma, max_newton=steps, eps_kkt=0.0, cg_max=4)
    Pi = torch.empty((inst.M, inst.N), dtype=torch.float64, device=dev)
    hist = np.zeros(steps + 1)
    r = pb.newton(Pi, max_newton=steps, eps_kkt=0.0, cg_max=4, history=hist)
    assert (r["stage1_iters"], r["stage2_iters"]) == (ref.stage1_iters, ref.stage2_iters)
    assert r["cg_iters"] == ref.cg_iters
    assert np.max(np.abs(Pi.cpu().numpy() - ref.X)) <= 1e-9
    n = len(ref.history)
    assert np.allclose(hist[:n], ref.history, rtol=1e-10, atol=0)
    assert r["objective"] == pytest.approx(ref.f, rel=1e-10)
    pb.close()


def test_c1_solve_reaches_the_certified_optimum(dev):
    inst, F, pb = setup("c1")
    with open(os.path.join(GOLDEN, "c1_oracle.json")) as fh:
        gold = json.load(fh)
    fstar = gold["f_star"]
    ref = newton.two_stage(F, inst.P, inst.gamma, max_newton=200, eps_kkt=1e-13)
    Pi = torch.empty((inst.M, inst.N), dtype=torch.float64, device=dev)
    hist = np.zeros(201)
    r = pb.newton(Pi, max_newton=200, eps_kkt=1e-13, history=hist)
    X = Pi.cpu().numpy()
    print(f"[newton] c1 gpu {r} oracle f {ref.f} s1 {ref.stage1_iters} s2 {ref.stage2_iters}", flush=True)
    n = 1 + r["stage1_iters"] + r["stage2_iters"]
    assert np.all(np.diff(hist[:n]) <= 0)
    assert (ref.f - fstar) <= 1e-8 * fstar
    assert (r["objective"] - fstar) <= 1e-8 * fstar and r["objective"] >= fstar * (1 - 1e-13)
    assert np.max(np.abs(X - np.array(gold["Pi_star"]))) <= 1e-4
    assert np.all(X >= 0) and np.max(np.abs(X.sum(axis=1) - 1)) <= 1e-13
    assert r["kkt"] == pytest.approx(certify.kkt_residual(F, inst.P, X, inst.gamma, clamp=True), rel=1e-6, abs=1e-15)
    pb.close()


def test_stage2_only_and_user_start(dev):
    inst, F, pb = setup("small")
    ref = newton.two_stage(F, inst.P, inst.gamma, max_newton=4, eps_kkt=0.0, stage2_only=True, cg_max=4)
    Pi = torch.empty((inst.M, inst.N), dtype=torch.float64, device=dev)
    r = pb.newton(Pi, max_newton=4, eps_kkt=0.0, stage2_only=True, cg_max=4)
    assert r["stage1_iters"] == 0 and r["stage2_iters"] == ref.stage2_iters
    assert np.max(np.abs(Pi.cpu().numpy() - ref.X)) <= 1e-9
    # a user start is projected onto the simplex rows first
    X0 = np.random.default_rng(5).random((inst.M, inst.N)) * 3.0
    ref = newton.two_stage(F, inst.P, inst.gamma, max_newton=2, eps_kkt=0.0, X0=X0, cg_max=4)
    Pi = gpu(X0, dev)
    r = pb.newton(Pi, max_newton=2, eps_kkt=0.0, init=_pdt.PDT_INIT_USER, cg_max=4)
    assert np.max(np.abs(Pi.cpu().numpy() - ref.X)) <= 1e-9
    pb.close()


def test_invalid_options_are_rejected(dev):
    inst, F, pb = setup("ragged")
    Pi = torch.empty((inst.M, inst.N), dtype=torch.float64, device=dev)
    for kw in (dict(cg_max=0), dict(eps_kkt=-1.0), dict(max_newton=-1), dict(init=_pdt.PDT_INIT_LEARNED),
               dict(cg_rtol=float("nan"))):
        with pytest.raises(_pdt.PdtError) as ei:
            pb.newton(Pi, **kw)
        assert ei.value.status == _pdt.PDT_ERR_INVALID_ARG
    with pytest.raises(_pdt.PdtError):
        pb.newton_direction(3, Pi, 0.0, 1e-4, 10, Pi)
    # zero steps: the start is returned with its objective and a not-converged status
    r = pb.newton(Pi, max_newton=0)
    assert r["status"] == _pdt.PDT_ERR_NOT_CONVERGED
    assert np.allclose(Pi.cpu().numpy(), 1.0 / inst.N, rtol=0, atol=1e-16)
    pb.close()


def test_c2_full_size_steps(dev):
    """M=4096, N=65, D=5000 in the launch configuration of the benchmark: sampled Hessian
    rows against the oracle's row-at-a-time products, two whole Newton steps (4 CG
    iterations each) against the oracle, then 60 paper-default steps that decrease f
    monotonically and keep every row on the simplex."""
    inst = synth.c2_medium()
    pb = _pdt.Problem.from_instance(inst)
    ro = sampled.RowOracle(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    rows = [0, 1, 17, 640, 2047, 3001, 4094, 4095]
    V = np.random.default_rng(8).normal(size=(inst.M, inst.N))
    HV = torch.empty((inst.M, inst.N), dtype=torch.float64, device=dev)
    pb.hessian(gpu(V, dev), HV)
    ref_rows = ro.gradient_rows(np.zeros_like(inst.P), V, inst.gamma, rows)
    assert np.max(np.abs(HV.cpu().numpy()[rows] - ref_rows)) <= 1e-12 * np.max(np.abs(ref_rows))

    F, _, _ = poisson.build_F(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    print("[newton] c2 oracle, 2 steps", flush=True)
    ref = newton.two_stage(F, inst.P, inst.gamma, max_newton=2, eps_kkt=0.0, cg_max=4)
    Pi = torch.empty((inst.M, inst.N), dtype=torch.float64, device=dev)
    r = pb.newton(Pi, max_newton=2, eps_kkt=0.0, cg_max=4)
    assert (r["stage1_iters"], r["cg_iters"]) == (ref.stage1_iters, ref.cg_iters)
    assert np.max(np.abs(Pi.cpu().numpy() - ref.X)) <= 1e-9
    assert r["objective"] == pytest.approx(ref.f, rel=1e-10)

    hist = np.zeros(61)
    r = pb.newton(Pi, max_newton=60, eps_kkt=0.0, history=hist)
    print(f"[newton] c2 60 steps {r}", flush=True)
    n = 1 + r["stage1_iters"] + r["stage2_iters"]
    assert np.all(np.diff(hist[:n]) <= 0) and hist[n - 1] < 1e-6 * hist[0]
    X = Pi.cpu().numpy()
    assert np.all(X >= 0) and np.max(np.abs(X.sum(axis=1) - 1)) <= 1e-12
    pb.close()
