"""Euclidean projection onto the probability simplex (App. B.1, two-stage extension).

P_S[x] = argmin_{y in S} ||x - y||_2,  S = {y : y_i >= 0, sum_i y_i = 1},
and its M-fold version P_{S^M} that projects every row of Pi on its own (Eq. Mp1_proj).

``project_simplex`` is the sort-based exact method (Held, Wolfe and Crowder 1974; in
the form of Duchi et al. 2008): with u sorted descending and c_j = sum_{k<=j} u_k, the
support size is rho = max{j : u_j - (c_j - 1)/j > 0}, the threshold is
tau = (c_rho - 1)/rho and P_S[x] = max(x - tau, 0).

``project_simplex_bruteforce`` enumerates every support S: the candidate is x shifted
by tau_S = (sum_S x - 1)/|S| on S and zero elsewhere; among the candidates that are
non-negative (points of the simplex) the nearest one to x is the projection, because
the projection lies in the relative interior of exactly one face.
"""
from __future__ import annotations

import itertools

import numpy as np


def simplex_threshold_rows(X: np.ndarray) -> np.ndarray:
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    n = X.shape[1]
    u = -np.sort(-X, axis=1)
    c = np.cumsum(u, axis=1)
    j = np.arange(1, n + 1, dtype=np.float64)
    cond = u - (c - 1.0) / j > 0
    rho = n - np.argmax(cond[:, ::-1], axis=1)  # last True, 1-based
    tau = (c[np.arange(X.shape[0]), rho - 1] - 1.0) / rho
    return tau


def project_rows(X: np.ndarray) -> np.ndarray:
    """P_{S^M}: each row onto the simplex (Eq. Mp1_proj)."""
    X = np.atleast_2d(np.asarray(X, dtype=np.float64))
    tau = simplex_threshold_rows(X)
    return np.maximum(X - tau[:, None], 0.0)


def project_simplex(x: np.ndarray) -> np.ndarray:
    return project_rows(np.asarray(x, dtype=np.float64)[None, :])[0]


def project_simplex_bruteforce(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    best, best_d = None, np.inf
    for size in range(1, n + 1):
        for S in itertools.combinations(range(n), size):
            S = list(S)
            tau = (x[S].sum() - 1.0) / size
            y = np.zeros(n)
            y[S] = x[S] - tau
            if np.all(y[S] >= 0.0):
                dist = float(np.sum((x - y) ** 2))
                if dist < best_d:
                    best, best_d = y, dist
    return best
