"""Two-stage two-metric projected truncated Newton method (App. B, Algorithms 1-3).

The paper's own solver, written out from its description:

Stage 1 (Algorithm 2).  At Pi (rows on the simplex) with gradient g = grad f(Pi):
  * binding set I = {(i, n): Pi[i][n] <= eps and g[i][n] > 0}  (Eq. 2metric_I);
  * D = the Hessian on the free entries, its diagonal on I, and no coupling between
    I and the rest (the two-metric matrix D^(k) of App. B);
  * solve D P = -g by conjugate gradients preconditioned with the Hessian diagonal;
  * line search alpha = beta^l on Pi(alpha) = P_{S^M}[Pi + alpha P], accepting the first
    alpha with f(Pi(alpha)) <= f(Pi) + c alpha phi'(0), phi(alpha) = f(Pi(alpha))
    (Armijo, beta = 3/4, c = 1/10);
  * switch to stage 2 once |phi'(0)| <= 1e-4.

Stage 2 (Algorithm 1).  In every row the largest entry m(i) is eliminated through the
sum constraint, Pi[i][m(i)] = 1 - sum_{n != m(i)} Pi[i][n]; the remaining entries only
carry bounds >= 0.  With the chain rule the reduced gradient is g[i][n] - g[i][m(i)],
the reduced Hessian is T^T H T (T maps the reduced variables to Pi), and the same
two-metric step is taken with the bound projection max(., 0); a trial is accepted when
Armijo holds and every eliminated entry is >= 0.  Stops when the KKT residual with the
clamped multipliers of App. B falls below eps_kkt.

The Hessian of f is I_N (x) A with A = 2 F^T F + 2 gamma L (columns decouple), so its
diagonal is the per-row h_m of fista.hessian_diag and the reduced diagonal is 2 h_i.

Readings where the paper is silent (also listed in the design notes):
  * eps of the binding set ("a small eps"): Bertsekas's rule eps = min(cap, w) with
    cap = 1e-9 and w the norm of the projected-gradient residual: ||Pi - P_{S^M}[Pi - g]||
    in stage 1, and ||min(Pi, g_reduced)|| over the reduced variables in stage 2.  (A
    cap of 1e-3 binds POVM entries that are legitimately ~1e-4 at the optimum; on the
    M=4096 detector it left 800 Newton steps at 6.5e-4 relative, against 6.6e-6.);
  * CG: from P = 0, stops at ||r|| <= cg_rtol ||rhs|| (1e-4) or after cg_max (50) steps;
  * phi'(0) is the exact one-sided derivative at alpha = 0.  In stage 1, for a row x on
    the simplex, P_S(x + alpha d) = max(x + alpha d - alpha t, 0) for small alpha > 0,
    where t solves sum_{x_n > 0} (d_n - t) + sum_{x_n = 0} max(d_n - t, 0) = 0; the
    path's derivative is v_n = d_n - t on the support and max(d_n - t, 0) off it (the
    projection of d onto the tangent cone of the simplex at x).  In stage 2 the bound
    projection moves entry (i, n) by P unless Pi[i][n] = 0 and P < 0.  (A difference
    quotient carries rounding noise of ~1e-7 of X per entry at alpha = 1e-9, which
    decides the stage switch once |phi'(0)| is small.);
  * a direction that is not a descent direction (phi'(0) >= 0) is replaced by -g;
  * at most 60 line-search trials (beta^60 ~ 3e-8);
  * a zero Hessian diagonal entry (a row no probe reaches, gamma = 0) is taken as 1 in
    the preconditioner and in the diagonal block of the bound entries;
  * stage2_only=True starts in stage 2 (the comparison of App. B's convergence study).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .certify import kkt_residual
from .fista import hessian_apply, hessian_diag
from .objective import gradient, objective
from .simplex import project_rows

BETA = 0.75
C_ARMIJO = 0.1
EPS_CAP = 1e-9
MAX_TRIALS = 60


def pcg(apply_D, rhs: np.ndarray, diag: np.ndarray, rtol: float, max_iter: int):
    """Preconditioned CG for D P = rhs from P = 0; returns (P, iterations)."""
    P = np.zeros_like(rhs)
    r = rhs.copy()
    nr0 = math.sqrt(float(np.sum(rhs * rhs)))
    if nr0 == 0.0:
        return P, 0
    z = r / diag
    p = z.copy()
    rz = float(np.sum(r * z))
    it = 0
    for it in range(1, max_iter + 1):
        q = apply_D(p)
        pq = float(np.sum(p * q))
        if pq <= 0.0:
            break
        a = rz / pq
        P = P + a * p
        r = r - a * q
        if math.sqrt(float(np.sum(r * r))) <= rtol * nr0:
            break
        z = r / diag
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return P, it


def stage1_direction(F, gamma: float, Pi: np.ndarray, g: np.ndarray, h: np.ndarray, eps: float,
                     rtol: float, max_iter: int):
    """Two-metric Newton direction on the simplex rows (Algorithm 2)."""
    bind = (Pi <= eps) & (g > 0)
    free = ~bind
    hd = np.broadcast_to(np.where(h > 0, h, 1.0)[:, None], Pi.shape)

    def apply_D(v):
        return np.where(free, hessian_apply(F, gamma, np.where(free, v, 0.0)), 0.0) + np.where(bind, hd * v, 0.0)

    P, it = pcg(apply_D, -g, hd, rtol, max_iter)
    return P, it, bind


def tangent_direction(x: np.ndarray, d: np.ndarray) -> np.ndarray:
    """d/dalpha P_S(x + alpha d) at alpha = 0+ for one row x on the simplex: the shift t
    over the support and the zero entries whose d_n exceeds it, found by growing the
    threshold until the set of entries above it stops changing (each pass can only
    drop entries, so it ends after at most N passes)."""
    zero = x == 0.0
    active = np.ones(x.shape, dtype=bool)
    while True:
        t = float(np.sum(d[active])) / int(np.count_nonzero(active))
        keep = ~zero | (d > t)
        if np.array_equal(keep & active, active):
            break
        active &= keep
    return np.where(zero, np.maximum(d - t, 0.0), d - t)


def stage1_slope(Pi: np.ndarray, P: np.ndarray, g: np.ndarray) -> float:
    v = np.stack([tangent_direction(Pi[i], P[i]) for i in range(Pi.shape[0])])
    return float(np.sum(g * v))


def reduce_max(Pi: np.ndarray) -> np.ndarray:
    """m(i) = argmax_n Pi[i][n], lowest index on ties (Algorithm 1)."""
    return np.argmax(Pi, axis=1)


def expand(v: np.ndarray, mi: np.ndarray) -> np.ndarray:
    """T v: reduced variables (zero at m(i)) to a change of Pi that keeps row sums."""
    u = v.copy()
    rows = np.arange(v.shape[0])
    u[rows, mi] = 0.0
    u[rows, mi] = -u.sum(axis=1)
    return u


def contract(w: np.ndarray, mi: np.ndarray) -> np.ndarray:
    """T^T w: (T^T w)[i][n] = w[i][n] - w[i][m(i)] for n != m(i), 0 at m(i)."""
    rows = np.arange(w.shape[0])
    out = w - w[rows, mi][:, None]
    out[rows, mi] = 0.0
    return out


def stage2_direction(F, gamma: float, Pi: np.ndarray, g: np.ndarray, h: np.ndarray, eps: float,
                     rtol: float, max_iter: int):
    """Two-metric Newton direction in the reduced variables (Algorithm 1)."""
    M, N = Pi.shape
    mi = reduce_max(Pi)
    rows = np.arange(M)
    gr = contract(g, mi)
    var = np.ones(Pi.shape, dtype=bool)
    var[rows, mi] = False
    bind = var & (Pi <= eps) & (gr > 0)
    free = var & ~bind
    hd = np.broadcast_to(np.where(h > 0, 2.0 * h, 1.0)[:, None], Pi.shape)

    def apply_D(v):
        w = contract(hessian_apply(F, gamma, expand(np.where(free, v, 0.0), mi)), mi)
        return np.where(free, w, 0.0) + np.where(bind, hd * v, 0.0)

    P, it = pcg(apply_D, np.where(var, -gr, 0.0), np.where(var, hd, 1.0), rtol, max_iter)
    P = np.where(var, P, 0.0)
    return P, it, mi, bind


def stage2_trial(Pi: np.ndarray, P: np.ndarray, mi: np.ndarray, alpha: float):
    rows = np.arange(Pi.shape[0])
    X = np.maximum(Pi + alpha * P, 0.0)
    X[rows, mi] = 0.0
    X[rows, mi] = 1.0 - X.sum(axis=1)
    return X


def stage2_slope(Pi: np.ndarray, P: np.ndarray, g: np.ndarray, mi: np.ndarray) -> float:
    d = np.where((Pi > 0) | (P > 0), P, 0.0)
    return float(np.sum(g * expand(d, mi)))


@dataclasses.dataclass
class NewtonResult:
    X: np.ndarray
    f: float
    stage1_iters: int
    stage2_iters: int
    cg_iters: int
    history: list
    kkt: float


def binding_eps_stage1(Pi: np.ndarray, g: np.ndarray, cap: float = EPS_CAP) -> float:
    return min(cap, math.sqrt(float(np.sum((Pi - project_rows(Pi - g)) ** 2))))


def binding_eps_stage2(Pi: np.ndarray, g: np.ndarray, mi: np.ndarray, cap: float = EPS_CAP) -> float:
    v = np.minimum(Pi, contract(g, mi))
    v[np.arange(Pi.shape[0]), mi] = 0.0
    return min(cap, math.sqrt(float(np.sum(v * v))))


def two_stage(F, P: np.ndarray, gamma: float, *, max_newton: int = 200, eps_kkt: float = 1e-10,
              stage_switch: float = 1e-4, cg_rtol: float = 1e-4, cg_max: int = 50,
              X0: np.ndarray | None = None, stage2_only: bool = False, eps_cap: float = EPS_CAP) -> NewtonResult:
    M = F.shape[1]
    N = P.shape[1]
    X = project_rows(np.full((M, N), 1.0 / N) if X0 is None else X0)
    h = hessian_diag(F, gamma, M)
    f = objective(F, P, X, gamma, exact=False)
    hist = [f]
    stage = 2 if stage2_only else 1
    n1 = n2 = cg_total = 0
    for _ in range(max_newton):
        g = gradient(F, P, X, gamma)
        if stage == 2 and kkt_residual(F, P, X, gamma, clamp=True) <= eps_kkt:
            break
        if stage == 1:
            D, it, _ = stage1_direction(F, gamma, X, g, h, binding_eps_stage1(X, g, eps_cap), cg_rtol, cg_max)
            slope = stage1_slope(X, D, g)
            if slope >= 0.0:
                D = -g
                slope = stage1_slope(X, D, g)
            if abs(slope) <= stage_switch:
                stage = 2
                continue
            trial = lambda a: project_rows(X + a * D)  # noqa: E731
            ok = lambda Xa: True  # noqa: E731
            n1 += 1
        else:
            D, it, mi, _ = stage2_direction(F, gamma, X, g, h, binding_eps_stage2(X, g, reduce_max(X), eps_cap),
                                            cg_rtol, cg_max)
            slope = stage2_slope(X, D, g, mi)
            if slope >= 0.0:
                D = np.where(np.arange(N)[None, :] == mi[:, None], 0.0, -contract(g, mi))
                slope = stage2_slope(X, D, g, mi)
            if slope == 0.0:
                break
            trial = lambda a, D=D, mi=mi: stage2_trial(X, D, mi, a)  # noqa: E731
            ok = lambda Xa, mi=mi: bool(np.all(Xa[np.arange(M), mi] >= 0.0))  # noqa: E731
            n2 += 1
        cg_total += it
        a = 1.0
        accepted = False
        for _ in range(MAX_TRIALS):
            Xa = trial(a)
            if ok(Xa):
                fa = objective(F, P, Xa, gamma, exact=False)
                if fa <= f + C_ARMIJO * a * slope:
                    X, f = Xa, fa
                    accepted = True
                    break
            a *= BETA
        hist.append(f)
        if not accepted:
            if stage == 1:
                stage = 2
            else:
                break
    return NewtonResult(X=X, f=f, stage1_iters=n1, stage2_iters=n2, cg_iters=cg_total, history=hist,
                        kkt=kkt_residual(F, P, X, gamma, clamp=True))
