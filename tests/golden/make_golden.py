"""Writes the stored expected values under tests/golden/ by calling the CPU oracle only.

c1_oracle.json -- the M=64, N=9, D=80 workload (8-bin click detector, mu in [0, 40],
dense F, gamma = 1e-3): the oracle's Lipschitz estimate, its objective after 2000
iterations of the accelerated projected-gradient iteration from the uniform start, and
the exact optimum obtained by active-set polishing of a 20000-iteration run (certified
by the sign checks of the KKT conditions).

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import certify, fista, poisson  # noqa: E402
from paper_2404_02844_amd import synth  # noqa: E402


def main():
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


if __name__ == "__main__":
    main()
