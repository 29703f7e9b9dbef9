"""Learned warm start vs the cold start on the M=16384, N=129 detector family.

Family: click detectors with bins ~ U{8..128} (outcomes beyond bins+1 are zero columns),
efficiency ~ U(0.5, 0.95), dark counts ~ U(0, 1e-3) per bin, crosstalk ~ U(0, 0.02);
D = round(1.2 M) probes with mu linearly spaced to 1.1 M; 1e7 shots per probe;
gamma = 1e-4.  Training and test detectors come from disjoint seed streams.

Protocol per test detector: the cold FP64 solve, the warm FP64 solve and the warm mixed
solve (all with the row-scaled step), and the cold FP64 solve with the uniform step 1/L,
each run K iterations with the objective recorded after every iteration; the reference
optimum is the lowest objective any of them reached.  Iterations to a relative
objective tol are read from the histories; times are iterations x the run's measured
time per iteration, plus the measured cost of the learned start for warm runs.

Usage:  python -m paper_2404_02844_amd.experiments --out results.json
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

M_FAMILY = 16384
N_PAD = 129


def _gen(args):
    stream, i = args
    from paper_2404_02844_amd import synth
    rng = synth.rng_for(stream, spawn=i)
    return synth.random_detector(rng, M_FAMILY, bins=(8, 128), eta=(0.5, 0.95), dark=(0.0, 1e-3),
                                 crosstalk=(0.0, 0.02), n_pad_to=N_PAD, shots=1e7, gamma=1e-4,
                                 name=f"ws{stream}_{i}")


def generate(stream: int, count: int, workers: int):
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_gen, [(stream, i) for i in range(count)]))


def iters_to(hist: np.ndarray, fref: float, tol: float):
    ok = np.nonzero((hist - fref) <= tol * fref)[0]
    return int(ok[0]) + 1 if ok.size else None


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=96)
    ap.add_argument("--test", type=int, default=4)
    ap.add_argument("--target-iters", type=int, default=3000)
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--K", type=int, default=30000)
    ap.add_argument("--hidden", type=int, default=512)
    ap.add_argument("--uniform-tests", type=int, default=4,
                    help="test detectors that also run the uniform-step solve (it does not reach 1e-8 in K)")
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)

    import torch

    from paper_2404_02844_amd import _pdt, warmstart

    def log(*a):
        print(*a, flush=True)

    workers = min(16, os.cpu_count() or 1)
    t0 = time.time()
    train = generate(5, args.train, workers)
    test = generate(6, args.test, workers)
    log(f"[ws] generated {len(train)} + {len(test)} detectors in {time.time() - t0:.1f} s")

    t0 = time.time()
    pairs = []
    for k, inst in enumerate(train):
        pairs.append(warmstart.solve_pair(inst, max_iters=args.target_iters, precision=_pdt.PDT_MIXED))
        if k % 16 == 15:
            log(f"[ws] targets {k + 1}/{len(train)} ({time.time() - t0:.1f} s)")
    t_targets = time.time() - t0
    log(f"[ws] solver targets: {sum(p.X.shape[0] for p in pairs)} columns in {t_targets:.1f} s")

    sizes = [258, args.hidden, args.hidden, args.hidden, M_FAMILY]
    rng = np.random.default_rng(0)
    model = _pdt.Model(258, args.hidden, M_FAMILY, _pdt.pack_params(warmstart.init_layers(rng, sizes)))
    t0 = time.time()
    hist = warmstart.train(model, pairs, epochs=args.epochs, batch=256, lr=1e-3, lr_decay=0.985,
                           log_every=max(1, args.epochs // 10))
    t_train = time.time() - t0
    log(f"[ws] trained {model.num_params} parameters in {t_train:.1f} s, loss {hist[0]:.3e} -> {hist[-1]:.3e}")

    results = []
    for ti, inst in enumerate(test):
        pb = _pdt.Problem.from_instance(inst)
        runs = {}
        DIAG, UNIFORM = _pdt.PDT_STEP_DIAG, _pdt.PDT_STEP_UNIFORM
        # the scaled step's Lipschitz constant is set up once per problem, outside the timings
        pb.solve(torch.zeros((inst.M, inst.N), dtype=torch.float64, device="cuda"), max_iters=0, scaling=DIAG)
        plan = [("cold_fp64", _pdt.PDT_INIT_UNIFORM, _pdt.PDT_FP64, DIAG),
                ("warm_fp64", _pdt.PDT_INIT_LEARNED, _pdt.PDT_FP64, DIAG),
                ("warm_mixed", _pdt.PDT_INIT_LEARNED, _pdt.PDT_MIXED, DIAG)]
        if ti < args.uniform_tests:
            plan.append(("cold_fp64_uniform", _pdt.PDT_INIT_UNIFORM, _pdt.PDT_FP64, UNIFORM))
        for name, init, prec, sc in plan:
            Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device="cuda")
            h = torch.zeros(args.K, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t = time.time()
            info = pb.solve(Pi, init=init, precision=prec, max_iters=args.K, history=h, scaling=sc,
                            model=model if init == _pdt.PDT_INIT_LEARNED else None)
            torch.cuda.synchronize()
            wall = time.time() - t
            runs[name] = {"hist": h.cpu().numpy(), "wall": wall, "info": info}
        # cost of the learned start alone (features, network, projection, two evaluations)
        Pi = torch.zeros((inst.M, inst.N), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        t = time.time()
        f0 = pb.solve(Pi, init=_pdt.PDT_INIT_LEARNED, model=model, max_iters=0)
        torch.cuda.synchronize()
        t_init = time.time() - t
        t = time.time()
        c0 = pb.solve(Pi, max_iters=0)
        torch.cuda.synchronize()
        t_cold0 = time.time() - t
        fref = min(float(r["hist"].min()) for r in runs.values())
        row = {"bins": inst.detector["B"], "eta": inst.detector["eta"], "dark": inst.detector["dark"],
               "crosstalk": inst.detector["crosstalk"], "f_ref": fref,
               "f_start_cold": c0["objective"], "f_start_warm": f0["objective"],
               "fell_back": f0["fell_back_to_cold"], "learned_start_s": t_init - t_cold0}
        for name, r in runs.items():
            cold = name.startswith("cold")
            per_it = (r["wall"] - (t_cold0 if cold else t_init)) / args.K
            row[name] = {"s_per_iter": per_it, "wall": r["wall"], "final_relobj": (float(r["hist"][-1]) - fref) / fref}
            for tol in (1e-4, 1e-6, 1e-8):
                k = iters_to(r["hist"], fref, tol)
                extra = 0.0 if cold else row["learned_start_s"]
                row[name][f"iters_{tol:g}"] = k
                row[name][f"time_{tol:g}"] = None if k is None else k * per_it + extra
        log(f"[ws] test bins={row['bins']}: " + ", ".join(
            f"{n}: it1e-6={row[n]['iters_1e-06']} it1e-8={row[n]['iters_1e-08']}" for n in runs))
        results.append(row)
        pb.close()

    def med(key, tol):
        vals = [r[key][f"time_{tol:g}"] for r in results if key in r]
        vals = [v for v in vals if v is not None]
        return float(np.median(vals)) if vals else None

    def stats(vals, seed=0):
        """median, interquartile range and a 95% bootstrap interval of the median"""
        v = np.asarray(vals, dtype=np.float64)
        if v.size == 0:
            return None
        rng = np.random.default_rng(seed)
        boots = np.median(rng.choice(v, size=(2000, v.size), replace=True), axis=1)
        return {"n": int(v.size), "median": float(np.median(v)), "iqr": [float(np.percentile(v, 25)), float(np.percentile(v, 75))],
                "ci95_median": [float(np.percentile(boots, 2.5)), float(np.percentile(boots, 97.5))]}

    summary = {"family": f"M={M_FAMILY} N={N_PAD} D=19661", "train_detectors": args.train,
               "train_columns": int(sum(p.X.shape[0] for p in pairs)), "target_iters": args.target_iters,
               "epochs": args.epochs, "hidden": args.hidden, "train_loss": [hist[0], hist[-1]],
               "t_targets_s": t_targets, "t_train_s": t_train, "K": args.K, "tests": results}
    for tol in (1e-4, 1e-6, 1e-8):
        summary[f"median_time_{tol:g}"] = {k: med(k, tol) for k in ("cold_fp64", "warm_fp64", "warm_mixed",
                                                                    "cold_fp64_uniform")}
        summary[f"median_iters_{tol:g}"] = {
            k: (float(np.median([r[k][f"iters_{tol:g}"] for r in results
                                 if k in r and r[k][f"iters_{tol:g}"] is not None]))
                if any(k in r and r[k][f"iters_{tol:g}"] is not None for r in results) else None)
            for k in ("cold_fp64", "warm_fp64", "warm_mixed", "cold_fp64_uniform")}
    for tol in (1e-6, 1e-8):
        key = f"{tol:g}"
        summary[f"stats_time_{key}"] = {k: stats([r[k][f"time_{key}"] for r in results if k in r and r[k][f"time_{key}"] is not None])
                                        for k in ("cold_fp64", "warm_fp64", "warm_mixed")}
        paired = [(r["cold_fp64"][f"iters_{key}"], r["warm_fp64"][f"iters_{key}"]) for r in results]
        summary[f"reached_{key}"] = {k: int(sum(1 for r in results if k in r and r[k][f"iters_{key}"] is not None))
                                     for k in ("cold_fp64", "warm_fp64", "warm_mixed", "cold_fp64_uniform")}
        summary[f"stats_iter_ratio_cold_over_warm_{key}"] = stats([c / w for c, w in paired if c and w])
    log(json.dumps({k: v for k, v in summary.items() if k != "tests"}, indent=1))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(summary, fh, indent=1, default=float)


if __name__ == "__main__":
    sys.exit(main())
