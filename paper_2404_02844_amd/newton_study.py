"""Studies of the paper's own solver on synthetic detectors (App. B and Sec. 3.2).

1. Two-stage vs stage-2-only convergence (the comparison of App. B's convergence
   figure, there on the experiment with gamma = 0): objective after each Newton step
   from Pi = 1/N, steps and time to a relative objective, for both starts.
2. Long-range smoothing restart (Sec. 3.2, Eq. smoothing): a two-stage solve from
   1/N, its result smoothed with N_smooth(i) = i / 50 (lowest 100 rows kept), then a
   stage-2-only solve from the smoothed start.  The synthetic detector's true POVM is
   known, so each result is scored by its mean fidelity to it (Eq. fidelities), and by
   its objective.
3. The momentum method (row-scaled step) on the same problem, to the same tolerance,
   for reference.
4. (--sweep) The stage-switch threshold, the CG budget per Newton step and the cap of
   the binding tolerance, varied around the paper's values (|phi'(0)| <= 1e-4, 50
   iterations) and the Bertsekas reading (cap 1e-3), 800 steps each.

Every solve runs in the HIP library; this module only sequences calls and scores.

    python -m paper_2404_02844_amd.newton_study --out newton_study.json
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import time

import numpy as np

from . import _pdt, synth


def fidelity_columns(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Eq. fidelities for diagonal POVM elements, one value per outcome column."""
    num = np.sum(np.sqrt(np.clip(A, 0, None) * np.clip(B, 0, None)), axis=0) ** 2
    den = A.sum(axis=0) * B.sum(axis=0)
    out = np.ones(A.shape[1])
    ok = den > 0
    out[ok] = num[ok] / den[ok]
    return out


def rel_steps(hist: np.ndarray, f_ref: float, tols=(1e-4, 1e-6, 1e-8)) -> dict:
    out = {}
    for t in tols:
        idx = np.flatnonzero(hist - f_ref <= t * f_ref)
        out[f"{t:g}"] = int(idx[0]) if idx.size else None
    return out


def run(inst, dev, max_newton: int, eps_kkt: float, log) -> dict:
    import torch
    pb = _pdt.Problem.from_instance(inst)
    M, N = inst.M, inst.N
    Pi = torch.empty((M, N), dtype=torch.float64, device=dev)
    res = {"workload": inst.name, "M": M, "N": N, "D": inst.D, "gamma": inst.gamma}
    # reference optimum from the row-scaled momentum method
    t = time.perf_counter()
    ref = pb.solve(Pi, max_iters=60000, scaling=_pdt.PDT_STEP_DIAG)
    torch.cuda.synchronize()
    f_ref = ref["objective"]
    res["reference"] = {"f": f_ref, "kkt": ref["kkt"], "iters": ref["iters"], "time_s": time.perf_counter() - t}
    log(f"[study] {inst.name} gamma={inst.gamma}: reference f={f_ref:.12e} kkt={ref['kkt']:.2e}")
    for tol in (1e-6, 1e-9):
        t = time.perf_counter()
        r = pb.solve(Pi, max_iters=60000, scaling=_pdt.PDT_STEP_DIAG, f_star=f_ref, rel_obj_tol=tol)
        torch.cuda.synchronize()
        res[f"momentum_{tol:g}"] = {"iters": r["iters"], "time_s": time.perf_counter() - t,
                                    "converged": r["converged"]}
    for name, s2 in (("two_stage", False), ("stage2_only", True)):
        hist = np.zeros(max_newton + 1)
        t = time.perf_counter()
        r = pb.newton(Pi, max_newton=max_newton, eps_kkt=eps_kkt, stage2_only=s2, history=hist)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        n = 1 + r["stage1_iters"] + r["stage2_iters"]
        h = hist[:n]
        res[name] = {"time_s": el, "stage1": r["stage1_iters"], "stage2": r["stage2_iters"], "cg": r["cg_iters"],
                     "trials": r["line_trials"], "kkt": r["kkt"], "relobj": (r["objective"] - f_ref) / f_ref,
                     "steps_to": rel_steps(h, f_ref), "history_relobj": ((h - f_ref) / f_ref).tolist()}
        for tol in (1e-6, 1e-9):
            t = time.perf_counter()
            r2 = pb.newton(Pi, max_newton=max_newton, eps_kkt=eps_kkt, stage2_only=s2, f_star=f_ref,
                           rel_obj_tol=tol)
            torch.cuda.synchronize()
            res[name][f"time_to_{tol:g}"] = time.perf_counter() - t if r2["converged"] else None
        log(f"[study] {name}: {res[name]['stage1']}+{res[name]['stage2']} steps, cg {res[name]['cg']}, "
            f"{el:.2f} s, relobj {res[name]['relobj']:.2e}, to 1e-6/1e-9: {res[name]['time_to_1e-06']} / "
            f"{res[name]['time_to_1e-09']} s")
    # smoothing restart: two-stage solve, smooth, stage-2-only solve
    r1 = pb.newton(Pi, max_newton=max_newton, eps_kkt=eps_kkt)
    X1 = Pi.cpu().numpy()
    Sm = _pdt.pdt_smooth_rows(Pi)
    torch.cuda.synchronize()
    Xs = Sm.cpu().numpy()
    f_s = pb.objective(Sm)
    r2 = pb.newton(Sm, max_newton=max_newton, eps_kkt=eps_kkt, init=_pdt.PDT_INIT_USER, stage2_only=True)
    X2 = Sm.cpu().numpy()
    fid = {k: float(np.mean(fidelity_columns(X, inst.Pi_true))) for k, X in
           (("first_run", X1), ("smoothed", Xs), ("second_run", X2))}
    fmin = {k: float(np.min(fidelity_columns(X, inst.Pi_true))) for k, X in
            (("first_run", X1), ("smoothed", Xs), ("second_run", X2))}
    res["smoothing_restart"] = {"f_first": r1["objective"], "f_smoothed": f_s, "f_second": r2["objective"],
                                "second_run_steps": r2["stage2_iters"], "mean_fidelity": fid, "min_fidelity": fmin}
    log(f"[study] smoothing restart: f {r1['objective']:.6e} -> smoothed {f_s:.6e} -> {r2['objective']:.6e}; "
        f"mean fidelity {fid}")
    pb.close()
    return res


def sweep(inst, dev, log) -> list:
    import torch
    pb = _pdt.Problem.from_instance(inst)
    Pi = torch.empty((inst.M, inst.N), dtype=torch.float64, device=dev)
    f_ref = pb.solve(Pi, max_iters=30000, scaling=_pdt.PDT_STEP_DIAG)["objective"]
    out = []
    grid = [(sw, cg, 1e-3) for sw in (1e-4, 1e-6, 1e-8, 0.0) for cg in (50, 20)]
    grid += [(sw, 50, cap) for sw in (1e-4, 0.0) for cap in (1e-4, 1e-6, 1e-9, 1e-14)]
    for switch, cg_max, cap in grid:
        if True:
            hist = np.zeros(801)
            t = time.perf_counter()
            r = pb.newton(Pi, max_newton=800, eps_kkt=0.0, stage_switch=switch, cg_max=cg_max, history=hist,
                          eps_cap=cap)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            n = 1 + r["stage1_iters"] + r["stage2_iters"]
            rec = {"stage_switch": switch, "cg_max": cg_max, "eps_cap": cap, "time_s": el, "stage1": r["stage1_iters"],
                   "stage2": r["stage2_iters"], "cg": r["cg_iters"], "trials": r["line_trials"],
                   "relobj": (r["objective"] - f_ref) / f_ref, "kkt": r["kkt"],
                   "steps_to": rel_steps(hist[:n], f_ref, (1e-1, 1e-2, 1e-3, 1e-4, 1e-6))}
            log(f"[sweep] switch {switch:g} cg {cg_max} eps cap {cap:g}: {rec['stage1']}+{rec['stage2']} steps {el:.2f} s "
                f"relobj {rec['relobj']:.2e} kkt {rec['kkt']:.2e} steps_to {rec['steps_to']}")
            out.append(rec)
    pb.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--max-newton", type=int, default=400)
    ap.add_argument("--eps-kkt", type=float, default=1e-12)
    ap.add_argument("--out", default="")
    ap.add_argument("--sweep", action="store_true", help="only the stage-switch / CG-budget sweep")
    args = ap.parse_args(argv)
    import torch
    dev = torch.device("cuda:0")

    def log(*a):
        print(*a, flush=True)

    if args.sweep:
        out = sweep(synth.c2_medium(), dev, log)
        if args.out:
            with open(args.out, "w") as fh:
                json.dump(out, fh)
        return out
    out = []
    for seed_off, gamma in ((0, 0.0), (0, 1e-4)):
        base = synth.c2_medium(seed_offset=seed_off)
        inst = dataclasses.replace(base, gamma=gamma, name=f"{base.name}_gamma{gamma:g}")
        out.append(run(inst, dev, args.max_newton, args.eps_kkt, log))
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh)
    return out


if __name__ == "__main__":
    main()
