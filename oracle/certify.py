"""Optimality certificates, the exact small-problem optimum, and POVM fidelity.

KKT residual (App. B, convergence criterion of the second stage):
    sqrt( (1/(N M)) sum_{i,n} (Pi_{i,n} (df/dPi_{i,n} + lambda_i))^2 ),
with the row multiplier estimate lambda_i = -min_n df/dPi_{i,n}.  The paper clamps it
at zero, lambda_i = max(0, -min_n df/dPi_{i,n}); the multiplier of an equality
constraint carries no sign, so the unclamped estimate is the default and the clamped
one is available with ``clamp=True``.

Frank-Wolfe gap (Jaggi 2013): sum_i (<grad_i, Pi_i> - min_n grad_{i,n}).  For a convex
f over a product of simplices it bounds f(Pi) - f* from above.

``polish`` solves the equality-constrained quadratic program on a fixed support S
exactly: with H = 2 F^T F + 2 gamma L applied per column, it solves
    [H_SS  A^T] [x     ]   [2 (F^T P)_S]
    [A     0  ] [lambda] = [1          ]
(A sums each row's support entries), and certifies the result as the optimum of the
full problem when x > 0 and the reduced gradient grad + lambda is >= 0 off S.

Fidelity of two diagonal POVM elements (Eq. fidelities): for commuting diagonal
pi and theta the matrix square roots are element-wise, so
    F = (sum_i sqrt(pi_i theta_i))^2 / (sum_i pi_i * sum_i theta_i).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .objective import gradient, objective


def kkt_residual(F, P, Pi, gamma, clamp: bool = False) -> float:
    G = gradient(F, P, Pi, gamma)
    lam = -G.min(axis=1)
    if clamp:
        lam = np.maximum(lam, 0.0)
    r = Pi * (G + lam[:, None])
    return math.sqrt(math.fsum((r * r).ravel()) / r.size)


def fw_gap(F, P, Pi, gamma) -> float:
    G = gradient(F, P, Pi, gamma)
    return math.fsum((np.sum(G * Pi, axis=1) - G.min(axis=1)).tolist())


@dataclasses.dataclass
class PolishResult:
    Pi: np.ndarray
    f: float
    certified: bool
    min_support_entry: float
    min_reduced_grad: float
    cond: float


def polish(F, P, Pi_approx, gamma, support_tol: float = 1e-9) -> PolishResult:
    Fd = F.toarray() if hasattr(F, "toarray") else np.asarray(F)
    M, N = Pi_approx.shape
    Hm = 2.0 * (Fd.T @ Fd)
    if M > 1:
        Lm = np.zeros((M, M))
        idx = np.arange(M - 1)
        Lm[idx, idx] += 1.0
        Lm[idx + 1, idx + 1] += 1.0
        Lm[idx, idx + 1] -= 1.0
        Lm[idx + 1, idx] -= 1.0
        Hm = Hm + 2.0 * gamma * Lm
    b_full = 2.0 * (Fd.T @ P)  # [M, N]
    S = [(i, n) for n in range(N) for i in range(M) if Pi_approx[i, n] > support_tol]
    ns = len(S)
    K = np.zeros((ns + M, ns + M))
    rhs = np.zeros(ns + M)
    for a, (i, n) in enumerate(S):
        for b, (j, m) in enumerate(S):
            if n == m:
                K[a, b] = Hm[i, j]
        K[a, ns + i] = 1.0
        K[ns + i, a] = 1.0
        rhs[a] = b_full[i, n]
    rhs[ns:] = 1.0
    sol = np.linalg.solve(K, rhs)
    Pi = np.zeros((M, N))
    for a, (i, n) in enumerate(S):
        Pi[i, n] = sol[a]
    G = gradient(F, P, Pi, gamma)
    lam = sol[ns:]
    red = G + lam[:, None]
    mask = np.ones((M, N), dtype=bool)
    for (i, n) in S:
        mask[i, n] = False
    min_entry = float(sol[:ns].min())
    min_red = float(red[mask].min()) if mask.any() else 0.0
    return PolishResult(Pi=Pi, f=objective(F, P, Pi, gamma), certified=(min_entry > 0 and min_red >= 0),
                        min_support_entry=min_entry, min_reduced_grad=min_red,
                        cond=float(np.linalg.cond(K)))


def fidelity(pi: np.ndarray, theta: np.ndarray) -> float:
    pi = np.asarray(pi, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    num = math.fsum(np.sqrt(np.maximum(pi, 0) * np.maximum(theta, 0)).tolist()) ** 2
    den = math.fsum(pi.tolist()) * math.fsum(theta.tolist())
    return num / den if den > 0 else float("nan")
