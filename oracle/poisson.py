"""Coherent-probe matrix F of Eq. Fmatrix, written out plainly in FP64.

F[d, i] = mu_d^i exp(-mu_d) / i!   for i in [0, M-1]   (Eq. Fmatrix, Sec. 2.2;
mu_d = |alpha_d|^2 is the probe's mean photon number).

The pmf is evaluated with Loader's saddle-point form (C. Loader, "Fast and accurate
computation of binomial probabilities", 2000):

    log p(m; mu) = -stirlerr(m) - bd0(m, mu) - log(2 pi m) / 2,   m >= 1,
    p(0; mu) = exp(-mu),

with stirlerr(n) = log n! - [(n + 1/2) log n - n + log(2 pi)/2] and the deviance
bd0(x, l) = x log(x / l) + l - x, both free of the catastrophic cancellation that
mu log mu - mu - lgamma(m + 1) suffers at large mu.  Every entry is evaluated on its
own (no recursion across entries).

Sparsity (Sec. 3.2, Data distribution): for large M each row of F is non-negligible
only in a band around mu_d.  ``band_edges`` keeps the entries with value >= tau.

Column M-1 (reading): the paper truncates the photon-number expansion at M-1.  With
``tail_mode == LUMP`` column M-1 instead holds P(X >= M-1), so that each row of F
sums to one; this is used where the probes' mean photon numbers reach past M.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import sparse

TRUNCATE = 0
LUMP = 1

_HALF_LOG_2PI = 0.5 * math.log(2.0 * math.pi)


def stirlerr(n) -> np.ndarray:
    """log n! minus its Stirling approximation, for integers n >= 1."""
    n = np.atleast_1d(np.asarray(n, dtype=np.float64))
    out = np.empty_like(n)
    small = n <= 15
    if small.any():
        ns = n[small]
        logfact = np.array([math.log(math.factorial(int(k))) for k in ns])
        out[small] = logfact - ((ns + 0.5) * np.log(ns) - ns + _HALF_LOG_2PI)
    big = ~small
    if big.any():
        r = 1.0 / n[big]
        r2 = r * r
        # Stirling series sum_k B_2k / (2k (2k-1) n^(2k-1)), k = 1..7:
        # 1/12n - 1/360n^3 + 1/1260n^5 - 1/1680n^7 + 1/1188n^9 - 691/360360n^11 + 1/156n^13
        inner = 1.0 / 1188 - r2 * (691.0 / 360360 - r2 / 156)
        out[big] = r * (1.0 / 12 - r2 * (1.0 / 360 - r2 * (1.0 / 1260 - r2 * (1.0 / 1680 - r2 * inner))))
    return out


def bd0(x, lam) -> np.ndarray:
    """x log(x/lam) + lam - x for x > 0, lam > 0 (series form where x ~ lam)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64), x.shape)
    d = x - lam
    s = x + lam
    out = np.empty_like(x)
    near = np.abs(d) < 0.1 * s
    far = ~near
    if far.any():
        out[far] = x[far] * np.log(x[far] / lam[far]) + lam[far] - x[far]
    if near.any():
        v = d[near] / s[near]
        acc = d[near] * v
        ej = 2.0 * x[near] * v
        v2 = v * v
        for j in range(1, 60):
            ej = ej * v2
            term = ej / (2 * j + 1)
            acc = acc + term
            if np.all(np.abs(term) <= 1e-18 * np.abs(acc)):
                break
        out[near] = acc
    return out


def log_pmf(m, mu: float) -> np.ndarray:
    """log Poisson(m; mu) for integer m >= 0 (Eq. Fmatrix)."""
    m = np.atleast_1d(np.asarray(m, dtype=np.float64))
    out = np.full(m.shape, -np.inf)
    if mu == 0.0:
        out[m == 0] = 0.0
        return out
    z = m == 0
    out[z] = -mu
    nz = ~z
    if nz.any():
        mm = m[nz]
        out[nz] = -stirlerr(mm) - bd0(mm, mu) - (_HALF_LOG_2PI + 0.5 * np.log(mm))
    return out


def pmf(m, mu: float) -> np.ndarray:
    return np.exp(log_pmf(m, mu))


def upper_tail(mu: float, k0: int) -> float:
    """P(X >= k0) for X ~ Poisson(mu), by exactly rounded summation of pmf terms."""
    if k0 <= 0:
        return 1.0
    if mu == 0.0:
        return 0.0
    sd = math.sqrt(mu)
    if k0 > mu:
        hi = int(math.ceil(max(k0, mu) + 45.0 * sd + 200))
        terms = pmf(np.arange(k0, hi + 1), mu)
        return math.fsum(terms)
    lo = max(0, int(math.floor(mu - 45.0 * sd - 200)))
    terms = pmf(np.arange(lo, k0), mu)
    return 1.0 - math.fsum(terms)


def row_values(mu: float, lo: int, hi: int, M: int, tail_mode: int) -> np.ndarray:
    """F[d, lo..hi] for probe mean mu."""
    vals = pmf(np.arange(lo, hi + 1), mu)
    if tail_mode == LUMP and hi == M - 1:
        vals[-1] = upper_tail(mu, M - 1)
    return vals


def _value(mu: float, m: int, M: int, tail_mode: int) -> float:
    if tail_mode == LUMP and m == M - 1:
        return upper_tail(mu, M - 1)
    return float(pmf(m, mu)[0])


def band_edges(mu: float, M: int, tau: float, tail_mode: int) -> tuple[int, int]:
    """First and last m in [0, M-1] with F[d, m] >= tau (tau <= 0: the whole row).

    Returns (lo, hi) with lo > hi when no entry reaches tau.
    """
    if tau <= 0.0:
        return 0, M - 1
    sd = math.sqrt(max(mu, 1.0))
    w_lo = max(0, int(math.floor(mu - 14.0 * sd - 60)))
    w_hi = min(M - 1, int(math.ceil(mu + 14.0 * sd + 60)))
    if w_lo > M - 1:
        # every photon number below M-1 lies more than 14 sd under the mean: only the
        # lumped last column can reach tau
        if tail_mode == LUMP and upper_tail(mu, M - 1) >= tau:
            return M - 1, M - 1
        return 1, 0
    ms = np.arange(w_lo, w_hi + 1)
    vals = pmf(ms, mu)
    if tail_mode == LUMP and w_hi == M - 1:
        vals[-1] = upper_tail(mu, M - 1)
    idx = np.nonzero(vals >= tau)[0]
    if tail_mode == LUMP and idx.size == 0 and upper_tail(mu, M - 1) >= tau:
        return M - 1, M - 1
    if idx.size == 0:
        return 1, 0
    lo, hi = int(ms[idx[0]]), int(ms[idx[-1]])
    # the window must bracket the band (the pmf is unimodal in m)
    if (idx[0] == 0 and w_lo > 0) or (idx[-1] == ms.size - 1 and w_hi < M - 1):
        raise RuntimeError("band window too narrow")
    if tail_mode == LUMP and hi < M - 1 and upper_tail(mu, M - 1) >= tau:
        hi = M - 1
    return lo, hi


def bands(mu: np.ndarray, M: int, tau: float, tail_mode: int) -> tuple[np.ndarray, np.ndarray]:
    lo = np.empty(mu.shape[0], dtype=np.int64)
    hi = np.empty(mu.shape[0], dtype=np.int64)
    for d, m_ in enumerate(mu):
        lo[d], hi[d] = band_edges(float(m_), M, tau, tail_mode)
    return lo, hi


def build_F(mu: np.ndarray, M: int, tau: float, tail_mode: int):
    """F as a CSR matrix (D x M) holding exactly the band entries; plus the band edges."""
    lo, hi = bands(mu, M, tau, tail_mode)
    D = mu.shape[0]
    indptr = np.zeros(D + 1, dtype=np.int64)
    cols, data = [], []
    for d in range(D):
        if lo[d] <= hi[d]:
            c = np.arange(lo[d], hi[d] + 1)
            v = row_values(float(mu[d]), int(lo[d]), int(hi[d]), M, tail_mode)
        else:
            c = np.zeros(0, dtype=np.int64)
            v = np.zeros(0)
        cols.append(c)
        data.append(v)
        indptr[d + 1] = indptr[d] + c.size
    F = sparse.csr_matrix((np.concatenate(data), np.concatenate(cols), indptr), shape=(D, M))
    return F, lo, hi


def dense_F(mu: np.ndarray, M: int, tau: float, tail_mode: int) -> np.ndarray:
    return build_F(mu, M, tau, tail_mode)[0].toarray()
