"""Training driver of the learned warm start (all arithmetic in libpdt's HIP kernels).

Training pairs come from the solver itself: for each synthetic detector the solver's
converged Pi* gives one target column per real outcome n (0..bins), and the feature
row of that outcome is built on the GPU by ``pdt_warmstart_features``.  The network is
trained with ``pdt_model_train_step`` (BF16 MFMA forward/backward, FP32 Adam).
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import _pdt

N_IN = 258


@dataclasses.dataclass
class Pair:
    X: "object"  # float32 GPU tensor [bins+1, 258]
    T: "object"  # float32 GPU tensor [bins+1, M]  (columns of Pi*)
    iters: int
    f: float


def solve_pair(inst, *, max_iters: int, precision=_pdt.PDT_MIXED, start_from_truth: bool = True,
               rel_tol: float = 0.0, f_star: float = 0.0, scaling: int = _pdt.PDT_STEP_DIAG) -> Pair:
    """Solve one training detector and return its (features, Pi* columns) pair.

    Starting from the generating POVM (known for synthetic detectors) only shortens the
    solve; the target is the solver's optimum either way."""
    import torch
    pb = _pdt.Problem.from_instance(inst)
    Pi = torch.as_tensor(inst.Pi_true if start_from_truth else np.zeros((inst.M, inst.N)),
                         dtype=torch.float64, device="cuda").contiguous()
    info = pb.solve(Pi, precision=precision, init=_pdt.PDT_INIT_USER if start_from_truth else _pdt.PDT_INIT_UNIFORM,
                    max_iters=max_iters, rel_obj_tol=rel_tol, f_star=f_star, scaling=scaling)
    bins = inst.detector["B"]
    X = torch.empty((bins + 1, N_IN), dtype=torch.float32, device="cuda")
    got = _pdt.pdt_warmstart_features(pb.handle, X)
    assert got == bins, (got, bins)
    T = Pi[:, : bins + 1].t().contiguous().to(torch.float32)
    pb.close()
    return Pair(X=X, T=T, iters=int(info["iters"]), f=float(info["objective"]))


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
