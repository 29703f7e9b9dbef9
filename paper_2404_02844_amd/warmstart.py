"""Learned warm start: the detector family, solver-generated training pairs, training, and
the stored network (all arithmetic in libpdt's HIP kernels).

Family (M=16384, N=129): click detectors with bins ~ U{8..128} (outcomes beyond bins+1
are zero columns), efficiency ~ U(0.5, 0.95), dark counts ~ U(0, 1e-3) per bin,
crosstalk ~ U(0, 0.02); D = round(1.2 M) = 19,661 probes with mu linearly spaced to
1.1 M; 1e7 shots per probe; gamma = 1e-4.  Training detectors come from seed stream 5,
test detectors from stream 6 (disjoint).

Training pairs come from the solver itself: each training detector is solved from the
cold start Pi = 1/N with the row-scaled step until its KKT residual is at most kkt_tol
(the converged Pi*); the optimum's column n (0..bins) is the target of outcome n, whose
feature row is built on the GPU by ``pdt_warmstart_features``.  The network is trained
with ``pdt_model_train_step`` (BF16 MFMA forward/backward, FP32 master weights, Adam).

The trained network is stored as BF16 weight matrices (the precision of its products)
and FP32 biases in an .npz file.

Train:  python -m paper_2404_02844_amd.warmstart --detectors 160 --out warmstart_c5.npz
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import dataclasses
import json
import multiprocessing
import os
import sys
import time

import numpy as np

from . import _pdt

N_IN = 258
M_FAMILY = 16384
N_PAD = 129
HIDDEN = 512
SIZES = (N_IN, HIDDEN, HIDDEN, HIDDEN, M_FAMILY)
TRAIN_STREAM = 5
TEST_STREAM = 6
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warmstart_c5.npz")


def family_detector(stream: int, i: int, M: int = M_FAMILY):
    """Detector i of seed stream `stream` of the warm-start family."""
    from . import synth
    rng = synth.rng_for(stream, spawn=i)
    return synth.random_detector(rng, M, bins=(8, 128), eta=(0.5, 0.95), dark=(0.0, 1e-3),
                                 crosstalk=(0.0, 0.02), n_pad_to=N_PAD, shots=1e7, gamma=1e-4,
                                 name=f"ws{stream}_{i}")


def _gen(args):
    return family_detector(*args)


def generate(stream: int, indices, workers: int = 16):
    """Family detectors of one stream, generated in parallel processes (CPU)."""
    indices = list(indices)
    if workers <= 1 or len(indices) <= 1:
        return [family_detector(stream, i) for i in indices]
    # fresh interpreters, never forks of a process that may already use the GPU
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn")) as ex:
        return list(ex.map(_gen, [(stream, i) for i in indices]))


@dataclasses.dataclass
class Pair:
    X: "object"  # float32 GPU tensor [bins+1, 258]
    T: "object"  # float32 GPU tensor [bins+1, M]  (columns of Pi*)
    iters: int
    f: float
    kkt: float


def solve_target(inst, *, kkt_tol: float, max_iters: int, precision=_pdt.PDT_MIXED,
                 scaling: int = _pdt.PDT_STEP_DIAG) -> Pair:
    """Solve one training detector from Pi = 1/N until its KKT residual is <= kkt_tol
    and return its (features, Pi* columns) pair."""
    import torch
    pb = _pdt.Problem.from_instance(inst)
    Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device="cuda")
    info = pb.solve(Pi, precision=precision, max_iters=max_iters, kkt_tol=kkt_tol, scaling=scaling)
    bins = inst.detector["B"]
    X = torch.empty((bins + 1, N_IN), dtype=torch.float32, device="cuda")
    got = _pdt.pdt_warmstart_features(pb.handle, X)
    assert got == bins, (got, bins)
    T = Pi[:, : bins + 1].t().contiguous().to(torch.float32)
    pb.close()
    return Pair(X=X, T=T, iters=int(info["iters"]), f=float(info["objective"]), kkt=float(info["kkt"]))


def init_layers(rng: np.random.Generator, sizes) -> list:
    """Initial weights W ~ N(0, 1/fan_in) ([out, in]) and zero biases."""
    return [(rng.normal(0.0, 1.0 / np.sqrt(fin), size=(fout, fin)), np.zeros(fout))
            for fin, fout in zip(sizes[:-1], sizes[1:])]


def train(model: "_pdt.Model", pairs, *, epochs: int, batch: int = 256, lr: float = 1e-3, seed: int = 0,
          lr_decay: float = 1.0, log_every: int = 0):
    """Adam over the rows of all pairs, shuffled every epoch; returns the loss history."""
    import torch
    X = torch.cat([p.X for p in pairs], dim=0)
    T = torch.cat([p.T for p in pairs], dim=0)
    n = X.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        losses = []
        for k in range(0, n, batch):
            idx = perm[k:k + batch]
            losses.append(model.train_step(X[idx].contiguous(), T[idx].contiguous(), lr))
        hist.append(float(np.mean(losses)))
        lr *= lr_decay
        if log_every and (ep % log_every == 0 or ep == epochs - 1):
            print(f"[warmstart] epoch {ep} loss {hist[-1]:.3e} ({time.time() - t0:.1f} s)", flush=True)
    return hist


def _bf16_bits(a: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit patterns, rounded to nearest even."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def _bf16_to_f32(bits: np.ndarray) -> np.ndarray:
    return (bits.astype(np.uint32) << 16).view(np.float32)


def save_params(path: str, params: np.ndarray, sizes=SIZES, meta: dict | None = None) -> None:
    """Weight matrices as BF16, biases as FP32 (the flat FP32 parameter layout of pdt.h)."""
    layers = _pdt.unpack_params(params, list(sizes))
    out = {"sizes": np.asarray(sizes, dtype=np.int64), "meta": np.asarray(json.dumps(meta or {}))}
    for li, (W, b) in enumerate(layers):
        out[f"W{li}"] = _bf16_bits(W.astype(np.float32))
        out[f"b{li}"] = b.astype(np.float32)
    np.savez_compressed(path, **out)


def load_params(path: str = WEIGHTS):
    """(flat FP32 parameter vector, sizes, meta) of a stored network."""
    with np.load(path, allow_pickle=False) as z:
        sizes = [int(v) for v in z["sizes"]]
        meta = json.loads(str(z["meta"]))
        layers = [(_bf16_to_f32(z[f"W{li}"]), z[f"b{li}"]) for li in range(len(sizes) - 1)]
    return _pdt.pack_params(layers), sizes, meta


def load_model(path: str = WEIGHTS, stream=None) -> "_pdt.Model":
    params, sizes, _ = load_params(path)
    return _pdt.Model(sizes[0], sizes[1], sizes[-1], params, stream=stream)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--detectors", type=int, default=160, help="training detectors (seed stream 5)")
    ap.add_argument("--kkt-tol", type=float, default=1e-12)
    ap.add_argument("--max-iters", type=int, default=30000)
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--budget-s", type=float, default=0.0, help="stop solving targets after this many seconds")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--log", default="")
    args = ap.parse_args(argv)
    import torch

    def log(*a):
        print(*a, flush=True)

    workers = min(16, os.cpu_count() or 1)
    t0 = time.time()
    pairs, stats = [], []
    block = 32
    pending = None
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=multiprocessing.get_context("spawn")) as ex:
        def submit(lo):
            hi = min(lo + block, args.detectors)
            return ex.map(_gen, [(TRAIN_STREAM, i) for i in range(lo, hi)]) if lo < hi else None
        pending = submit(0)
        lo = 0
        while pending is not None:
            insts = list(pending)
            lo += len(insts)
            pending = submit(lo)  # the next block is generated while this one is solved
            for inst in insts:
                p = solve_target(inst, kkt_tol=args.kkt_tol, max_iters=args.max_iters)
                pairs.append(p)
                stats.append({"bins": inst.detector["B"], "iters": p.iters, "kkt": p.kkt, "f": p.f})
                log(f"[warmstart] target {len(pairs)}/{args.detectors}: bins {inst.detector['B']} "
                    f"iterations {p.iters} KKT {p.kkt:.2e} ({time.time() - t0:.0f} s)")
                if args.budget_s and time.time() - t0 > args.budget_s:
                    break
            if args.budget_s and time.time() - t0 > args.budget_s:
                break
    t_targets = time.time() - t0
    rng = np.random.default_rng(0)
    model = _pdt.Model(N_IN, HIDDEN, M_FAMILY, _pdt.pack_params(init_layers(rng, SIZES)))
    t1 = time.time()
    hist = train(model, pairs, epochs=args.epochs, batch=256, lr=1e-3, lr_decay=0.985,
                 log_every=max(1, args.epochs // 10))
    t_train = time.time() - t1
    meta = {"family": f"M={M_FAMILY} N={N_PAD} D=19661, seed stream {TRAIN_STREAM}",
            "train_detectors": len(pairs), "train_columns": int(sum(p.X.shape[0] for p in pairs)),
            "targets": f"cold mixed-precision solve, row-scaled step, KKT residual <= {args.kkt_tol:g} "
                       f"(at most {args.max_iters} iterations)",
            "target_iters_median": float(np.median([s["iters"] for s in stats])),
            "target_kkt_max": float(max(s["kkt"] for s in stats)),
            "targets_unconverged": int(sum(1 for s in stats if s["kkt"] > args.kkt_tol)),
            "epochs": args.epochs, "batch": 256, "lr": 1e-3, "lr_decay": 0.985,
            "loss_first": hist[0], "loss_last": hist[-1], "t_targets_s": t_targets, "t_train_s": t_train}
    save_params(args.out, model.params(), SIZES, meta)
    log(json.dumps(meta, indent=1))
    if args.log:
        with open(args.log, "w") as fh:
            json.dump({"meta": meta, "targets": stats, "loss": hist}, fh, indent=1)


if __name__ == "__main__":
    sys.exit(main())
