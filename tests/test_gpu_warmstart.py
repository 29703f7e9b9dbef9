"""Learned warm start on the GPU: network kernels vs the FP64 oracle network, features vs
the oracle's resampling, Adam, fallback, and the gain over the cold start.

Tolerances for the BF16 network (products in BF16, FP32 accumulation): cosine >= 0.999
and relative L2 error <= 2e-2 per tensor against FP64.
"""
import numpy as np
import pytest

from oracle import mlp, simplex
from paper_2404_02844_amd import _pdt, synth, warmstart

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pdt.lib()
    return torch.device("cuda:0")


def close(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
    rel = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return cos, rel


def small_family(i, M=256, bins=(8, 16)):
    rng = synth.rng_for(60, spawn=i)
    return synth.random_detector(rng, M, bins=bins, n_pad_to=bins[1] + 1, crosstalk=(0.0, 0.02), shots=1e7,
                                 name=f"wsfam_{i}")


def test_features_match_oracle(dev):
    inst = small_family(0)
    pb = _pdt.Problem.from_instance(inst)
    B = inst.detector["B"]
    X = torch.empty((B + 1, 258), dtype=torch.float32, device=dev)
    assert _pdt.pdt_warmstart_features(pb.handle, X) == B
    ref = mlp.features(inst.mu, inst.P, B)
    assert np.max(np.abs(X.cpu().numpy() - ref)) <= 2e-7 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("sizes,B", [([258, 64, 64, 64, 300], 37), ([258, 128, 128, 128, 1000], 129)])
def test_forward_and_gradients_match_oracle(dev, sizes, B):
    rng = np.random.default_rng(sum(sizes) + B)
    layers = mlp.init_params(rng, sizes)
    layers = [(W, rng.normal(size=b.shape) * 0.05) for W, b in layers]
    model = _pdt.Model(sizes[0], sizes[1], sizes[-1], _pdt.pack_params(layers))
    # the GPU keeps FP32 master weights: compare against the oracle on the same values
    ref_layers = _pdt.unpack_params(model.params(), sizes)
    X = rng.normal(size=(B, sizes[0])) * 0.5
    Xg = torch.as_tensor(X, dtype=torch.float32, device=dev)
    Y = model.forward(Xg).cpu().numpy()
    Yr, cache = mlp.forward(ref_layers, X.astype(np.float32).astype(np.float64))
    cos, rel = close(Y, Yr)
    assert cos >= 0.999 and rel <= 2e-2, (cos, rel)
    dY = rng.normal(size=Yr.shape) / Yr.size
    grads = model.gradients(Xg, torch.as_tensor(dY, dtype=torch.float32, device=dev)).cpu().numpy()
    gref = mlp.backward(ref_layers, cache, dY)
    got = _pdt.unpack_params(grads, sizes)
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(got, gref)):
        for name, a, b in (("W", gW, rW), ("b", gb, rb)):
            cos, rel = close(a, b)
            assert cos >= 0.999 and rel <= 2e-2, (li, name, cos, rel)


def test_adam_step_and_loss_decrease(dev):
    sizes = [258, 64, 64, 64, 200]
    rng = np.random.default_rng(3)
    model = _pdt.Model(258, 64, 200, _pdt.pack_params(mlp.init_params(rng, sizes)))
    X = torch.as_tensor(rng.normal(size=(50, 258)) * 0.5, dtype=torch.float32, device=dev)
    T = torch.as_tensor(rng.random(size=(50, 200)), dtype=torch.float32, device=dev)
    p0 = model.params()
    Y = model.forward(X)
    dY = 2.0 * (Y - T) / Y.numel()
    g = model.gradients(X, dY).cpu().numpy()
    lr = 1e-3
    model.train_step(X, T, lr)
    p1 = model.params()
    # the first Adam step moves each weight by lr * g / (|g| + 1e-8 / ...) -> lr * sign(g)
    big = np.abs(g) > 1e-5
    assert np.allclose((p0 - p1)[big], lr * np.sign(g[big]), rtol=2e-3, atol=1e-7)
    losses = [model.train_step(X, T, lr) for _ in range(60)]
    assert losses[-1] < 0.5 * losses[0]


def test_fallback_to_cold_start(dev):
    inst = small_family(1)
    rng = np.random.default_rng(9)
    sizes = [258, 32, 32, 32, inst.M]
    bad = [(W * 50.0, b + 30.0) for W, b in mlp.init_params(rng, sizes)]
    model = _pdt.Model(258, 32, inst.M, _pdt.pack_params(bad))
    pb = _pdt.Problem.from_instance(inst)
    Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
    info = pb.solve(Pi, init=_pdt.PDT_INIT_LEARNED, model=model, max_iters=50)
    cold = torch.zeros_like(Pi)
    info_c = pb.solve(cold, max_iters=50)
    if info["fell_back_to_cold"]:
        assert torch.equal(Pi, cold)
    else:  # the (projected) prediction was at least as good as 1/N
        assert info["objective"] <= info_c["objective"] * (1 + 1e-12) or info["iters"] == 50
    # a model of the wrong output size is rejected
    wrong = _pdt.Model(258, 32, inst.M + 1)
    with pytest.raises(_pdt.PdtError):
        pb.solve(Pi, init=_pdt.PDT_INIT_LEARNED, model=wrong, max_iters=5)


def test_learned_start_small_family(dev):
    """Train on converged solver outputs of 24 small detectors, test on 3 unseen ones: the
    learned start has a lower objective than Pi = 1/N, and both starts reach a relative
    objective of 1e-4 (reference optimum from a long cold solve).  The iteration counts
    are printed, not asserted: the momentum method's count is set by the slowest modes of
    the problem, which a better start need not shorten (at M=16384 the measured
    cold/warm time ratio is about 1)."""
    M = 256
    train_pairs = [warmstart.solve_target(small_family(i, M), kkt_tol=1e-12, max_iters=20000,
                                          precision=_pdt.PDT_FP64) for i in range(2, 26)]
    rng = np.random.default_rng(0)
    model = _pdt.Model(258, 128, M, _pdt.pack_params(mlp.init_params(rng, [258, 128, 128, 128, M])))
    hist = warmstart.train(model, train_pairs, epochs=300, batch=128, lr=1e-3)
    assert hist[-1] < 0.2 * hist[0]
    gains = []
    for i in range(100, 103):
        inst = small_family(i, M)
        pb = _pdt.Problem.from_instance(inst)
        Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
        f_cold0 = pb.solve(Pi, max_iters=0)["objective"]
        f_warm0 = pb.solve(Pi, init=_pdt.PDT_INIT_LEARNED, model=model, max_iters=0)["objective"]
        assert f_warm0 < f_cold0
        ref = pb.solve(Pi, max_iters=40000)
        fstar = ref["objective"]
        Pi.zero_()
        cold = pb.solve(Pi, max_iters=40000, rel_obj_tol=1e-4, f_star=fstar)
        Pi.zero_()
        warm = pb.solve(Pi, init=_pdt.PDT_INIT_LEARNED, model=model, max_iters=40000, rel_obj_tol=1e-4, f_star=fstar)
        assert warm["converged"] == 1 and cold["converged"] == 1
        assert warm["fell_back_to_cold"] == 0
        gains.append(cold["iters"] / max(warm["iters"], 1))
        print(f"[warmstart small] detector {i}: f(start) cold {f_cold0:.4e} learned {f_warm0:.4e}; "
              f"iterations to 1e-4 cold {cold['iters']} learned {warm['iters']}", flush=True)


# ---- the M=16384, N=129 network (258 -> 512 -> 512 -> 512 -> 16384) --------------------

C5_SIZES = [258, 512, 512, 512, 16384]


def test_c5_network_matches_oracle(dev):
    rng = np.random.default_rng(16384)
    layers = mlp.init_params(rng, C5_SIZES)
    layers = [(W, rng.normal(size=b.shape) * 0.05) for W, b in layers]
    model = _pdt.Model(258, 512, 16384, _pdt.pack_params(layers))
    ref_layers = _pdt.unpack_params(model.params(), C5_SIZES)
    B = 129
    X = np.concatenate([rng.random(size=(B, 256)) * 0.02, rng.random(size=(B, 2))], axis=1)
    Xg = torch.as_tensor(X, dtype=torch.float32, device=dev)
    Y = model.forward(Xg).cpu().numpy()
    Yr, cache = mlp.forward(ref_layers, X.astype(np.float32).astype(np.float64))
    cos, rel = close(Y, Yr)
    print(f"[c5 network] forward cos={cos:.6f} rel={rel:.2e}", flush=True)
    assert cos >= 0.999 and rel <= 2e-2, (cos, rel)
    dY = rng.normal(size=Yr.shape) / Yr.size
    grads = model.gradients(Xg, torch.as_tensor(dY, dtype=torch.float32, device=dev)).cpu().numpy()
    gref = mlp.backward(ref_layers, cache, dY)
    for li, ((gW, gb), (rW, rb)) in enumerate(zip(_pdt.unpack_params(grads, C5_SIZES), gref)):
        for name, a, b in (("W", gW, rW), ("b", gb, rb)):
            cos, rel = close(a, b)
            print(f"[c5 network] layer {li} d{name} cos={cos:.6f} rel={rel:.2e}", flush=True)
            assert cos >= 0.999 and rel <= 2e-2, (li, name, cos, rel)


@pytest.fixture(scope="module")
def c5_model(dev):
    import os
    if not os.path.exists(warmstart.WEIGHTS):
        pytest.fail(f"{warmstart.WEIGHTS} is missing")
    return warmstart.load_model()


@pytest.fixture(scope="module")
def c5_test_detectors():
    return warmstart.generate(warmstart.TEST_STREAM, range(2), workers=2)


def test_c5_learned_start_matches_oracle(dev, c5_model, c5_test_detectors):
    # features -> network -> columns -> row projection, each stage against the oracle
    params, sizes, _ = warmstart.load_params()
    ref_layers = _pdt.unpack_params(params, sizes)
    for inst in c5_test_detectors:
        B = inst.detector["B"]
        pb = _pdt.Problem.from_instance(inst)
        Xf = torch.empty((B + 1, 258), dtype=torch.float32, device=dev)
        assert _pdt.pdt_warmstart_features(pb.handle, Xf) == B
        feats = mlp.features(inst.mu, inst.P, B)
        assert np.max(np.abs(Xf.cpu().numpy() - feats)) <= 2e-7 * max(1.0, np.max(np.abs(feats)))
        Y = c5_model.forward(Xf).cpu().numpy()
        Yr, _ = mlp.forward(ref_layers, Xf.cpu().numpy().astype(np.float64))
        cos, rel = close(Y, Yr)
        print(f"[c5 start] bins={B} network cos={cos:.6f} rel={rel:.2e}", flush=True)
        assert cos >= 0.999 and rel <= 2e-2, (cos, rel)
        Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
        info = pb.solve(Pi, init=_pdt.PDT_INIT_LEARNED, model=c5_model, max_iters=0)
        cols = np.zeros((inst.M, inst.N))
        cols[:, : B + 1] = Y.T.astype(np.float64)
        start = simplex.project_rows(cols)
        if info["fell_back_to_cold"]:
            assert np.all(Pi.cpu().numpy() == 1.0 / inst.N)
        else:
            assert np.max(np.abs(Pi.cpu().numpy() - start)) <= 1e-12
            # and the oracle's own start (FP64 network) is as close as BF16 products allow
            cols[:, : B + 1] = Yr.T
            cos, rel = close(Pi.cpu().numpy(), simplex.project_rows(cols))
            assert cos >= 0.999 and rel <= 2e-2, (cos, rel)
        pb.close()


@pytest.mark.timeout(400)
def test_c5_learned_start_measured(dev, c5_model, c5_test_detectors):
    """Unseen detectors of the M=16384 family: the trained network's start is accepted (its
    objective lies below that of Pi = 1/N), and the warm and cold solves reach the same
    optimum; the iterations each needs to relative objectives of 1e-2 and 1e-8 are
    reported, not asserted (the measured gain is none: see the warm-start results)."""
    for inst in c5_test_detectors:
        pb = _pdt.Problem.from_instance(inst)
        Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device=dev)
        fstar = pb.solve(Pi, precision=_pdt.PDT_MIXED, max_iters=40000, kkt_tol=1e-13,
                         scaling=_pdt.PDT_STEP_DIAG)["objective"]
        Pi.zero_()
        start = pb.solve(Pi, init=_pdt.PDT_INIT_LEARNED, model=c5_model, max_iters=0)
        assert start["fell_back_to_cold"] == 0
        assert start["objective"] < pb.solve(torch.zeros_like(Pi), max_iters=0)["objective"]
        out = {}
        for name, init in (("cold", _pdt.PDT_INIT_UNIFORM), ("warm", _pdt.PDT_INIT_LEARNED)):
            for tol in (1e-2, 1e-8):
                Pi.zero_()
                out[name, tol] = pb.solve(Pi, init=init, model=c5_model if init else None, precision=_pdt.PDT_MIXED,
                                          max_iters=40000, rel_obj_tol=tol, f_star=fstar, scaling=_pdt.PDT_STEP_DIAG)
        print(f"[c5 gain] bins={inst.detector['B']} iterations to 1e-2: cold {out['cold', 1e-2]['iters']} "
              f"warm {out['warm', 1e-2]['iters']}; to 1e-8: cold {out['cold', 1e-8]['iters']} "
              f"warm {out['warm', 1e-8]['iters']}", flush=True)
        for tol in (1e-2, 1e-8):
            assert out["warm", tol]["converged"] == 1 and out["cold", tol]["converged"] == 1
        pb.close()
