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

Gradient restart (optional, restart="gradient"): the adaptive restart of O'Donoghue and
Candes (2015), in its gradient form.  After an accepted step the momentum is also reset
(t = 1, so the next beta is 0) when the step X' - X_k points against the gradient-mapping
direction Y - X', measured in the metric of the step (the variables W^{-1/2} Pi of the
row-scaled step):

    sum_m (1 / w_m) sum_n (Y - X')[m, n] (X' - X_k)[m, n] > 0.

The reject-and-reset of a step that raises f stays as it is.

L_hat = 1.05 * lambda_max(2 F^T F + 2 gamma L), lambda_max from 100 power iterations
started at the unit vector 1/sqrt(M): lambda_k = ||H v_{k-1}||, v_k = H v_{k-1} / lambda_k.

Row-scaled step (optional).  The paper preconditions its CG solves with the diagonal
of the Hessian (Table "ops": diagonal of the Hessian; App. B).  For this objective
that diagonal does not depend on the outcome column:

    h_m = 2 sum_d F[d][m]^2 + 2 gamma L[m][m]        (L[m][m] = 1 at the ends, 2 inside)

so a step scaled by 1/h_m per row of Pi keeps the constraint structure: each row is
scaled uniformly, and the projection in the metric diag(h) onto the product of row
simplices is still the row-wise Euclidean projection.  The step becomes
X' = P_{S^M}(Y - diag(w) G / L_w) with w_m = 1/max(h_m, 1e-12 max h) and
L_w = 1.05 * lambda_max(W^{1/2} H W^{1/2}) from the same 100-step power iteration
(the momentum method run in the variables W^{-1/2} Pi).
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


def hessian_diag(F, gamma: float, M: int) -> np.ndarray:
    """h_m = 2 sum_d F[d][m]^2 + 2 gamma L[m][m] (the Hessian diagonal, per row)."""
    Fd = F.toarray() if hasattr(F, "toarray") else np.asarray(F)
    ldiag = np.zeros(M)
    if M >= 2:
        ldiag[:] = 2.0
        ldiag[0] = ldiag[-1] = 1.0
    return np.array([2.0 * math.fsum(Fd[:, m] ** 2) for m in range(M)]) + 2.0 * gamma * ldiag


def row_weights(F, gamma: float, M: int) -> np.ndarray:
    """w_m = 1 / max(h_m, 1e-12 max_m h_m); all ones when h vanishes."""
    h = hessian_diag(F, gamma, M)
    hmax = float(np.max(h)) if M else 0.0
    if hmax <= 0.0:
        return np.ones(M)
    return 1.0 / np.maximum(h, 1e-12 * hmax)


def lipschitz_scaled(F, gamma: float, M: int, w: np.ndarray, iters: int = 100,
                     safety: float = 1.05) -> float:
    """1.05 * lambda_max(W^{1/2} H W^{1/2}) by power iteration from 1/sqrt(M)."""
    sw = np.sqrt(w)
    v = np.full(M, 1.0 / math.sqrt(M))
    lam = 0.0
    for _ in range(iters):
        z = sw * hessian_apply(F, gamma, sw * v)
        lam = math.sqrt(math.fsum(z * z))
        if lam == 0.0:
            break
        v = z / lam
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
            f_star: float | None = None, rel_tol: float | None = None,
            row_w: np.ndarray | None = None, restart: str = "function") -> FistaResult:
    """row_w: per-row step weights w (the step of row m is w_m / L_hat); None: w = 1.
    restart: "function" (reject a step that raises f and reset) or "gradient" (also reset
    the momentum after an accepted step that fails the gradient test)."""
    if restart not in ("function", "gradient"):
        raise ValueError(restart)
    M = F.shape[1]
    N = P.shape[1]
    X = project_rows(np.full((M, N), 1.0 / N) if X0 is None else X0)
    s = 1.0 / L_hat if row_w is None else (np.asarray(row_w, dtype=np.float64) / L_hat)[:, None]
    inv_w = np.ones((M, 1)) if row_w is None else 1.0 / np.asarray(row_w, dtype=np.float64)[:, None]

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
            reset = restart == "gradient" and float(np.sum(inv_w * (Y - Xn) * (Xn - X))) > 0.0
            Xp, Op = X, O
            X, O, f = Xn, On, fn
            t = 1.0 if reset else tn
        hist[k] = f
        k_done = k + 1
        if f_star is not None and rel_tol is not None and (f - f_star) <= rel_tol * f_star:
            break
    return FistaResult(X=X, f=f, iters=k_done, history=hist[:k_done], rejects=rejects, L_hat=L_hat)
