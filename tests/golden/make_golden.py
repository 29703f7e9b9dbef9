"""Writes the stored expected values under tests/golden/ by calling the CPU oracle only.

c1_oracle.json -- the M=64, N=9, D=80 workload (8-bin click detector, mu in [0, 40],
dense F, gamma = 1e-3): the oracle's Lipschitz estimate, its objective after 2000
iterations of the accelerated projected-gradient iteration from the uniform start, and
the exact optimum obtained by active-set polishing of a 20000-iteration run (certified
by the sign checks of the KKT conditions).

c2_oracle.json -- the M=4096, N=65, D=5000 workload (64-bin detector, mu in [0, 4500],
band threshold 1e-16, lumped tail, gamma = 1e-4): the row-scaled iteration (step w_m /
L_w) from the uniform start, run for 40000 iterations with F as a dense matrix (the
library's matrix product on all cores; about 30 minutes).  Stored: L_w, the objective
after selected iteration counts, the optimum's objective with its KKT residual and
Frank-Wolfe gap (f - f* <= gap), and a compact record of the optimum and of the
2000-iteration iterate: every 64th row, and the column and row sums.

Run from the repository root:  python tests/golden/make_golden.py [c1|c2]
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import certify, fista, poisson  # noqa: E402
from paper_2404_02844_amd import synth  # noqa: E402


def c1():
    inst = synth.c1_small()
    F, lo, hi = poisson.build_F(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    L = fista.lipschitz(F, inst.gamma, inst.M)
    r = fista.fista_r(F, inst.P, inst.gamma, L, 2000)
    r_long = fista.fista_r(F, inst.P, inst.gamma, L, 20000, exact_sums=False)
    pol = certify.polish(F, inst.P, r_long.X, inst.gamma, 1e-7)
    out = {
        "workload": inst.name,
        "L_hat": L,
        "f_2000": r.f,
        "rejects_2000": r.rejects,
        "f_star": pol.f,
        "polish_certified": bool(pol.certified),
        "polish_min_support_entry": pol.min_support_entry,
        "polish_min_reduced_grad": pol.min_reduced_grad,
        "Pi_star": pol.Pi.tolist(),
    }
    with open(os.path.join(HERE, "c1_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print({k: v for k, v in out.items() if k != "Pi_star"})


C2_MARKS = (100, 200, 500, 1000, 2000, 5000, 10000, 20000, 30000, 40000)
C2_ROW_STEP = 64


def c2(iters: int = 40000):
    import time

    import numpy as np

    t0 = time.time()
    inst = synth.c2_medium()
    F, _, _ = poisson.build_F(inst.mu, inst.M, inst.threshold, inst.tail_mode)
    Fd = F.toarray()
    w = fista.row_weights(Fd, inst.gamma, inst.M)
    Lw = fista.lipschitz_scaled(Fd, inst.gamma, inst.M, w)
    print(f"c2: set-up {time.time() - t0:.0f} s, L_w = {Lw!r}", flush=True)
    r2k = fista.fista_r(Fd, inst.P, inst.gamma, Lw, 2000, exact_sums=False, row_w=w)
    print(f"c2: 2000 iterations f = {r2k.f!r} ({time.time() - t0:.0f} s)", flush=True)
    r = fista.fista_r(Fd, inst.P, inst.gamma, Lw, iters, exact_sums=False, row_w=w)
    kkt = certify.kkt_residual(Fd, inst.P, r.X, inst.gamma)
    gap = certify.fw_gap(Fd, inst.P, r.X, inst.gamma)
    print(f"c2: {iters} iterations f = {r.f!r} kkt = {kkt:.3e} fw gap = {gap:.3e} ({time.time() - t0:.0f} s)",
          flush=True)
    rows = list(range(0, inst.M, C2_ROW_STEP))

    def record(X):
        return {"rows": X[rows].tolist(), "col_sums": X.sum(0).tolist(),
                "row_sum_dev": float(np.max(np.abs(X.sum(1) - 1.0)))}

    out = {
        "workload": inst.name,
        "step": "row-scaled (w_m / L_w)",
        "L_w": Lw,
        "iters": r.iters,
        "rejects": r.rejects,
        "f_at": {str(k): float(r.history[k - 1]) for k in C2_MARKS if k <= r.iters},
        "f_star": r.f,
        "kkt": kkt,
        "fw_gap": gap,
        "row_step": C2_ROW_STEP,
        "Pi_star": record(r.X),
        "Pi_2000": record(r2k.X),
    }
    with open(os.path.join(HERE, "c2_oracle.json"), "w") as fh:
        json.dump(out, fh)
    print({k: v for k, v in out.items() if not k.startswith("Pi_")})


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "c1"
    {"c1": c1, "c2": c2}[which]()
