"""Accelerated projected gradient with function restart, and the Lipschitz estimate.

The paper's solver (App. B, Algorithms 1-3) is a projected truncated-Newton method;
its first stage steps along a direction, projects row-wise onto the simplex with
P_{S^M} and accepts by a sufficient-decrease test.  The iteration here is that
stage's first-order analogue with Nesterov momentum (Beck and Teboulle 2009) and a
monotone reject-and-reset restart:

    t' = (1 + sqrt(1 + 4 t^2)) / 2,   beta = (t - 1) / t'
    Y  = X_k + beta (X_k - X_{k-1})
    G  = grad f(Y) = 2 F^T (F Y - P) + 2 gamma L Y
    X' = P_{S^M}(Y - G / L_hat)
    accept X' if f(X') <= f(X_k) (then t = t'), else keep X_k and reset t = 1.

F Y is formed from the stored products as F X_k + beta (F X_k - F X_{k-1}) (F is
linear), exactly as it is written in the definition of the iteration; F X' is a
fresh product.  After a reset beta = 0, so the next step is a plain projected
gradient step of length 1/L_hat, which decreases f when L_hat >= lambda_max.

L_hat = 1.05 * lambda_max(2 F^T F + 2 gamma L), lambda_max from 100 power iterations
started at the unit vector 1/sqrt(M): lambda_k = ||H v_{k-1}||, v_k = H v_{k-1} / lambda_k.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .objective import laplacian, regulariser, sum_squares
from .simplex import project_rows


def hessian_apply(F, gamma: float, v: np.ndarray) -> np.ndarray:
    return 2.0 * (F.T @ (F @ v)) + 2.0 * gamma * laplacian(v)


def lipschitz(F, gamma: float, M: int, iters: int = 100, safety: float = 1.05) -> float:
    v = np.full(M, 1.0 / math.sqrt(M))
    lam = 0.0
    for _ in range(iters):
        w = hessian_apply(F, gamma, v)
        lam = math.sqrt(math.fsum(w * w))
        if lam == 0.0:
            break
        v = w / lam
    return safety * lam


@dataclasses.dataclass
class FistaResult:
    X: np.ndarray
    f: float
    iters: int
    history: np.ndarray  # f after every iteration (accepted value)
    rejects: int
    L_hat: float


def fista_r(F, P: np.ndarray, gamma: float, L_hat: float, iters: int,
            X0: np.ndarray | None = None, exact_sums: bool = True,
            f_star: float | None = None, rel_tol: float | None = None) -> FistaResult:
    M = F.shape[1]
    N = P.shape[1]
    X = project_rows(np.full((M, N), 1.0 / N) if X0 is None else X0)
    s = 1.0 / L_hat

    def fval(O, Xc):
        return sum_squares(O - P, exact_sums) + regulariser(Xc, gamma, exact_sums)

    O = F @ X
    Xp, Op = X, O
    f = fval(O, X)
    t = 1.0
    hist = np.empty(iters)
    rejects = 0
    k_done = 0
    for k in range(iters):
        tn = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
        beta = (t - 1.0) / tn
        Y = X + beta * (X - Xp)
        OY = O + beta * (O - Op)
        G = 2.0 * (F.T @ (OY - P)) + 2.0 * gamma * laplacian(Y)
        Xn = project_rows(Y - s * G)
        On = F @ Xn
        fn = fval(On, Xn)
        if fn > f:
            Xp, Op = X, O
            t = 1.0
            rejects += 1
        else:
            Xp, Op = X, O
            X, O, f = Xn, On, fn
            t = tn
        hist[k] = f
        k_done = k + 1
        if f_star is not None and rel_tol is not None and (f - f_star) <= rel_tol * f_star:
            break
    return FistaResult(X=X, f=f, iters=k_done, history=hist[:k_done], rejects=rejects, L_hat=L_hat)
