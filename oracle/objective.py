"""Objective and gradient of the regularised least-squares problem.

f(Pi) = ||F Pi - P||_F^2 + gamma * sum_n sum_{i=0}^{M-2} (Pi_{i,n} - Pi_{i+1,n})^2

(Eq. min_obj2 with the squared two-norm, plus the nearest-neighbour term of
Eq. regul).  Its gradient is

grad f = 2 F^T (F Pi - P) + 2 gamma L Pi,

where L is the Laplacian of the path graph on photon numbers 0..M-1:
(L Y)_0 = Y_0 - Y_1, (L Y)_i = 2 Y_i - Y_{i-1} - Y_{i+1}, (L Y)_{M-1} = Y_{M-1} - Y_{M-2}.

F may be a dense ndarray or a scipy sparse matrix.  ``exact=True`` sums the squares
with ``math.fsum`` (exactly rounded sum of the individually rounded squares).
"""
from __future__ import annotations

import math

import numpy as np


def sum_squares(A: np.ndarray, exact: bool = True) -> float:
    a = np.asarray(A, dtype=np.float64).ravel()
    sq = a * a
    return math.fsum(sq) if exact else float(np.sum(sq))


def regulariser(Pi: np.ndarray, gamma: float, exact: bool = True) -> float:
    """gamma * sum (Pi_{i,n} - Pi_{i+1,n})^2 (Eq. regul)."""
    if gamma == 0.0 or Pi.shape[0] < 2:
        return 0.0
    return gamma * sum_squares(Pi[:-1] - Pi[1:], exact)


def laplacian(Y: np.ndarray) -> np.ndarray:
    """L Y for the path-graph Laplacian along axis 0."""
    out = np.zeros_like(Y)
    if Y.shape[0] < 2:
        return out
    diff = Y[:-1] - Y[1:]  # Y_i - Y_{i+1}
    out[:-1] += diff
    out[1:] -= diff
    return out


def residual(F, P: np.ndarray, Pi: np.ndarray) -> np.ndarray:
    return F @ Pi - P


def objective(F, P: np.ndarray, Pi: np.ndarray, gamma: float, exact: bool = True) -> float:
    return sum_squares(residual(F, P, Pi), exact) + regulariser(Pi, gamma, exact)


def gradient(F, P: np.ndarray, Pi: np.ndarray, gamma: float) -> np.ndarray:
    R = residual(F, P, Pi)
    return 2.0 * (F.T @ R) + 2.0 * gamma * laplacian(Pi)
