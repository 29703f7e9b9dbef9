"""Seeded synthetic inputs for phase-insensitive detector tomography.

Produces what a tomography experiment hands the solver -- probe mean photon numbers
mu_d and measured outcome frequencies P[d, n] -- together with the known detector
POVM Pi_true that generated them.  Nothing here implements the reconstruction: the
forward model used to sample P calls ``scipy.stats.poisson`` (a library routine), so
this module shares no arithmetic with either the CPU oracle or the HIP kernels.  Both
sides receive the same arrays from here.

Detector model (a click detector with B bins, outcome n = number of clicked bins,
N = B + 1 outcomes; the paper's detector is a multiplexed click counter, Sec. 2.2):

* dark counts: each bin clicks by itself with probability ``dark``; the chain of
  clicked-bin counts starts from Binomial(B, dark);
* every incident photon is detected with probability ``eta`` and lands in a
  uniformly chosen bin, so k clicked bins become k + 1 with probability
  eta * (B - k) / B;
* optional crosstalk: each primary click triggers each of its two neighbours with
  probability x if that neighbour is idle, modelled at the count level as
  k -> min(B, k + Binomial(2k, x (B - k) / (B - 1))).

Probe states are coherent states with mean photon numbers mu_d on a linear grid
(Eq. Fmatrix gives their photon-number distribution, a Poisson pmf).  Outcome
frequencies are multinomial samples of q_d = sum_m Poisson(m; mu_d) Pi_true[m, :]
with a fixed number of shots per probe.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy import stats

SEED_BASE = 240402844

TRUNCATE = 0  # F_{d,m} = Poisson(m; mu_d) for m < M (Eq. Fmatrix as printed)
LUMP = 1  # as TRUNCATE, but column M-1 carries the whole tail P(X >= M-1)


@dataclasses.dataclass
class Instance:
    """One tomography problem: inputs (mu, P, gamma, ...) plus the generating POVM."""

    name: str
    M: int
    N: int
    D: int
    mu: np.ndarray  # [D] float64, non-decreasing
    P: np.ndarray  # [D, N] float64, rows sum to 1
    Pi_true: np.ndarray  # [M, N] float64, rows on the simplex
    gamma: float
    tail_mode: int
    threshold: float  # pmf threshold tau of the F band (0 -> dense)
    shots: float
    seed: int
    detector: dict


def rng_for(k: int, spawn: Optional[int] = None) -> np.random.Generator:
    """PCG64 stream for config index k (and optionally its spawn-th child)."""
    ss = np.random.SeedSequence(SEED_BASE + k)
    if spawn is not None:
        ss = ss.spawn(spawn + 1)[spawn]
    return np.random.Generator(np.random.PCG64(ss))


def _chain_matrix(B: int, eta: float) -> np.ndarray:
    """One-photon transition matrix of the clicked-bin count (row-stochastic)."""
    k = np.arange(B + 1, dtype=np.float64)
    up = eta * (B - k) / B
    T = np.diag(1.0 - up)
    T[np.arange(B), np.arange(1, B + 1)] = up[:B]
    return T


def _crosstalk_matrix(B: int, x: float) -> np.ndarray:
    C = np.zeros((B + 1, B + 1))
    for k in range(B + 1):
        if k == 0 or x <= 0.0 or B < 2:
            C[k, k] = 1.0
            continue
        p = x * (B - k) / (B - 1)
        j = np.arange(2 * k + 1)
        w = stats.binom.pmf(j, 2 * k, p)
        for jj, ww in zip(j, w):
            C[k, min(B, k + jj)] += ww
    return C


def click_detector_povm(M: int, B: int, eta: float, dark: float = 0.0,
                        crosstalk: float = 0.0, block: int = 128) -> np.ndarray:
    """Pi_true[m, k] = P(k bins clicked | m photons), m in [0, M), k in [0, B]."""
    T = _chain_matrix(B, eta)
    pows = np.empty((block, B + 1, B + 1))
    pows[0] = np.eye(B + 1)
    for j in range(1, block):
        pows[j] = pows[j - 1] @ T
    step = pows[block - 1] @ T  # T^block
    out = np.empty((M, B + 1))
    row = stats.binom.pmf(np.arange(B + 1), B, dark) if dark > 0 else np.eye(B + 1)[0]
    for m0 in range(0, M, block):
        n = min(block, M - m0)
        out[m0:m0 + n] = np.einsum("k,jkl->jl", row, pows[:n])
        row = row @ step
    if crosstalk > 0:
        out = out @ _crosstalk_matrix(B, crosstalk)
    out = np.clip(out, 0.0, None)
    out /= out.sum(axis=1, keepdims=True)
    return out


LOOP_R, LOOP_ETA_LOOP, LOOP_ETA_DET = 0.91644, 0.90524, 0.528  # the paper's fitted device (Sec. 4.1)


def loop_bin_probs(J: int, R: float, eta_loop: float, eta_det: float) -> np.ndarray:
    """Per-photon click probability of time bins 1..J of the beam-splitter loop detector
    (the single-photon factors of Eq. pj_fock): R eta_det for the first bin, then
    (1 - R)^2 / R (R eta_loop)^(j-1) eta_det."""
    j = np.arange(1, J + 1, dtype=np.float64)
    q = (1.0 - R) ** 2 / R * (R * eta_loop) ** (j - 1.0) * eta_det
    q[0] = R * eta_det
    return q


_POOL_Q = None


def _loop_rows(args):
    i0, i1 = args
    q = _POOL_Q
    J = q.shape[0]
    i = np.arange(i0, i1, dtype=np.float64)[:, None]
    p = -np.expm1(i * np.log1p(-q)[None, :])  # p_j(i) = 1 - (1 - q_j)^i (Eq. pj_fock)
    dist = np.zeros((i1 - i0, J + 1))
    dist[:, 0] = 1.0
    for j in range(J):  # clicked-bin count, one independent bin at a time
        pj = p[:, j:j + 1]
        dist[:, 1:j + 2] = dist[:, 1:j + 2] * (1.0 - pj) + dist[:, 0:j + 1] * pj
        dist[:, 0] *= 1.0 - p[:, j]
    return dist


def loop_detector_povm(M: int, J: int = 150, R: float = LOOP_R, eta_loop: float = LOOP_ETA_LOOP,
                       eta_det: float = LOOP_ETA_DET, workers: int = 1, block: int = 4096) -> np.ndarray:
    """Pi_true[i, n] = P(n of the J time bins click | i photons) for the time-multiplexed
    loop detector of Sec. 4.1: bins click independently with p_j(i) = 1 - (1 - q_j)^i
    (Eq. pj_fock), so the count is Poisson-binomial; it is built by the exact one-bin-
    at-a-time recursion (data generation only).  Outcomes n = 0..J (N = J + 1)."""
    global _POOL_Q
    _POOL_Q = loop_bin_probs(J, R, eta_loop, eta_det)
    try:
        spans = [(i0, min(M, i0 + block)) for i0 in range(0, M, block)]
        if workers <= 1:
            parts = [_loop_rows(sp) for sp in spans]
        else:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(workers) as pool:
                parts = pool.map(_loop_rows, spans)
    finally:
        _POOL_Q = None
    out = np.concatenate(parts, axis=0)
    out = np.clip(out, 0.0, None)
    out /= out.sum(axis=1, keepdims=True)
    return out


def _probe_window(mu: float, lo_cap: int, hi_cap: int) -> tuple[int, int]:
    s = math.sqrt(max(mu, 1.0))
    lo = max(0, int(math.floor(mu - 12.0 * s - 40)))
    hi = min(hi_cap, int(math.ceil(mu + 12.0 * s + 40)))
    return max(lo, lo_cap), hi


_POOL_PI = None  # detector matrix inherited by forked generator processes


def _outcome_chunk(args):
    mu, M, tail_mode = args
    return _outcome_rows_blocked(mu, _POOL_PI, M, tail_mode)


def _outcome_rows_blocked(mu: np.ndarray, Pi_ext: np.ndarray, M: int, tail_mode: int, block: int = 64) -> np.ndarray:
    """LUMP rows for blocks of consecutive probes: one pmf matrix over the union of their
    windows and one matrix product per block, so Pi_true is streamed once per block."""
    D = mu.shape[0]
    N = Pi_ext.shape[1]
    q = np.zeros((D, N))
    for b0 in range(0, D, block):
        b1 = min(D, b0 + block)
        mus = mu[b0:b1].astype(np.float64)
        los, his = zip(*(_probe_window(float(m_), 0, M - 2) for m_ in mus))
        lo, hi = min(los), max(his)
        if lo <= hi:
            ms = np.arange(lo, hi + 1)
            W = stats.poisson.pmf(ms[None, :], mus[:, None])
            W[mus == 0.0] = 0.0
            W[mus == 0.0, 0] = 1.0 if lo == 0 else 0.0
            q[b0:b1] = W @ Pi_ext[lo:hi + 1]
        q[b0:b1] += stats.poisson.sf(M - 2, mus)[:, None] * Pi_ext[M - 1][None, :]
    return q


def outcome_probs(mu: np.ndarray, Pi_ext: np.ndarray, M: int, tail_mode: int, workers: int = 1) -> np.ndarray:
    """q_d = sum_m Poisson(m; mu_d) Pi_true[m, :] (scipy pmf; data generation only).

    LUMP: rows m >= M-1 of the detector are represented by row M-1 (tail mass on it).
    TRUNCATE: Pi_ext must extend far enough past M that the Poisson tail is negligible;
    the physical detector is defined for every photon number.  workers > 1 (LUMP only)
    splits the probes over forked processes and forms the rows of 64 consecutive probes
    with one matrix product over their joint window (the same sums, another rounding
    order).
    """
    if workers <= 1 or mu.shape[0] < 4 * workers or tail_mode != LUMP:
        q = _outcome_rows(mu, Pi_ext, M, tail_mode)
    else:
        import multiprocessing as mp
        global _POOL_PI
        _POOL_PI = Pi_ext
        try:
            # fixed 2048-probe chunks: the 64-probe blocks, and so the rounding, do not
            # depend on the number of workers
            chunks = [mu[k:k + 2048] for k in range(0, mu.shape[0], 2048)]
            with mp.get_context("fork").Pool(workers) as pool:
                q = np.concatenate(pool.map(_outcome_chunk, [(c, M, tail_mode) for c in chunks]), axis=0)
        finally:
            _POOL_PI = None
    q = np.clip(q, 0.0, None)
    return q / q.sum(axis=1, keepdims=True)


def _outcome_rows(mu: np.ndarray, Pi_ext: np.ndarray, M: int, tail_mode: int) -> np.ndarray:
    D = mu.shape[0]
    N = Pi_ext.shape[1]
    q = np.zeros((D, N))
    last = Pi_ext.shape[0] - 1
    for d in range(D):
        m_ = float(mu[d])
        if m_ == 0.0:
            q[d] = Pi_ext[0]
            continue
        if tail_mode == LUMP:
            lo, hi = _probe_window(m_, 0, M - 2)
            if lo <= hi:
                ms = np.arange(lo, hi + 1)
                q[d] = stats.poisson.pmf(ms, m_) @ Pi_ext[lo:hi + 1]
            q[d] += stats.poisson.sf(M - 2, m_) * Pi_ext[M - 1]
        else:
            lo, hi = _probe_window(m_, 0, last)
            ms = np.arange(lo, hi + 1)
            q[d] = stats.poisson.pmf(ms, m_) @ Pi_ext[lo:hi + 1]
    return q


def sample_outcomes(q: np.ndarray, shots: float, rng: np.random.Generator) -> np.ndarray:
    """P_d = Multinomial(shots, q_d) / shots."""
    counts = rng.multinomial(int(shots), q)
    return counts.astype(np.float64) / float(shots)


def make_instance(name: str, *, M: int, B: int, eta: float, D: int, mu_max: float,
                  shots: float, gamma: float, tail_mode: int, threshold: float,
                  dark: float = 0.0, crosstalk: float = 0.0,
                  rng: np.random.Generator, seed: int = 0, n_pad_to: Optional[int] = None,
                  noiseless: bool = False, workers: int = 1) -> Instance:
    N = B + 1
    mu = np.linspace(0.0, mu_max, D)
    if tail_mode == TRUNCATE:
        ext = int(math.ceil(mu_max + 14.0 * math.sqrt(max(mu_max, 1.0)) + 60))
        Pi_ext = click_detector_povm(max(M, ext + 1), B, eta, dark, crosstalk)
    else:
        Pi_ext = click_detector_povm(M, B, eta, dark, crosstalk)
    q = outcome_probs(mu, Pi_ext, M, tail_mode, workers=workers)
    P = q.copy() if noiseless else sample_outcomes(q, shots, rng)
    Pi_true = Pi_ext[:M].copy()
    if n_pad_to is not None and n_pad_to > N:
        P = np.concatenate([P, np.zeros((D, n_pad_to - N))], axis=1)
        Pi_true = np.concatenate([Pi_true, np.zeros((M, n_pad_to - N))], axis=1)
        N = n_pad_to
    return Instance(name=name, M=M, N=N, D=D, mu=mu, P=np.ascontiguousarray(P),
                    Pi_true=np.ascontiguousarray(Pi_true), gamma=gamma, tail_mode=tail_mode,
                    threshold=threshold, shots=shots, seed=seed,
                    detector=dict(B=B, eta=eta, dark=dark, crosstalk=crosstalk))


# --- the five workloads -------------------------------------------------------------

def c1_small(seed_offset: int = 0) -> Instance:
    """8-bin click detector, M=64, N=9, D=80 probes on mu in [0, 40], dense F."""
    return make_instance("c1_m64_n9_d80", M=64, B=8, eta=0.9, D=80, mu_max=40.0,
                         shots=1e6, gamma=1e-3, tail_mode=TRUNCATE, threshold=0.0,
                         rng=rng_for(1 + seed_offset), seed=SEED_BASE + 1 + seed_offset)


def c2_medium(seed_offset: int = 0) -> Instance:
    """64-bin detector, M=4096, N=65, D=5000 probes on mu in [0, 4500], band tau=1e-16."""
    return make_instance("c2_m4096_n65_d5000", M=4096, B=64, eta=0.85, dark=1e-4, D=5000,
                         mu_max=4500.0, shots=1e7, gamma=1e-4, tail_mode=LUMP, threshold=1e-16,
                         rng=rng_for(2 + seed_offset), seed=SEED_BASE + 2 + seed_offset)


def c3_mega(M: int = 1_000_000, D: int = 100_000, workers: int = 16) -> Instance:
    """99-bin detector with 1% crosstalk, M=1e6, N=100, D=1e5 probes on mu in [0, 1.1M]."""
    return make_instance(f"c3_m{M}_n100_d{D}", M=M, B=99, eta=0.8, crosstalk=0.01, D=D,
                         mu_max=1.1 * M, shots=1e8, gamma=1e-5, tail_mode=LUMP, threshold=1e-16,
                         rng=rng_for(3), seed=SEED_BASE + 3, workers=workers)


def loop_paper_scale(M: int = 1_210_581, D: int = 1076, J: int = 150, shots: float = 5e5, gamma: float = 1e-5,
                     workers: int = 16, seed_offset: int = 0) -> Instance:
    """The paper's experiment in synthetic form (Sec. 2.1, Sec. 4.1): the beam-splitter
    loop detector with its fitted R, eta_loop, eta_det, 150 time bins (N = 151), D = 1076
    coherent probes with mu_d = d^2, M = 1,210,581, 5e5 trials per probe, band tau = 1e-16
    (the probes' bands end below M - 1, so F is taken as printed, without a lumped tail)."""
    mu = np.arange(D, dtype=np.float64) ** 2
    ext = int(math.ceil(mu[-1] + 14.0 * math.sqrt(max(mu[-1], 1.0)) + 60))
    Pi_ext = loop_detector_povm(max(M, ext + 1), J, workers=workers)
    q = outcome_probs(mu, Pi_ext, M, TRUNCATE)
    P = sample_outcomes(q, shots, rng_for(6 + seed_offset))
    return Instance(name=f"loop_m{M}_n{J + 1}_d{D}", M=M, N=J + 1, D=D, mu=mu, P=np.ascontiguousarray(P),
                    Pi_true=np.ascontiguousarray(Pi_ext[:M]), gamma=gamma, tail_mode=TRUNCATE, threshold=1e-16,
                    shots=shots, seed=SEED_BASE + 6 + seed_offset,
                    detector=dict(kind="loop", J=J, R=LOOP_R, eta_loop=LOOP_ETA_LOOP, eta_det=LOOP_ETA_DET))


def random_detector(rng: np.random.Generator, M: int, *, bins=(8, 128), eta=(0.5, 0.95),
                    dark=(0.0, 1e-3), crosstalk=(0.0, 0.0), n_pad_to=None, shots=1e7,
                    gamma=1e-4, name="rand") -> Instance:
    """One detector of the batched / warm-start families (D = round(1.2 M), mu to 1.1 M)."""
    B = int(rng.integers(bins[0], bins[1] + 1))
    e = float(rng.uniform(*eta))
    dk = float(rng.uniform(*dark))
    xt = float(rng.uniform(*crosstalk)) if crosstalk[1] > 0 else 0.0
    D = int(round(1.2 * M))
    return make_instance(name, M=M, B=B, eta=e, dark=dk, crosstalk=xt, D=D, mu_max=1.1 * M,
                         shots=shots, gamma=gamma, tail_mode=LUMP, threshold=1e-16, rng=rng,
                         n_pad_to=n_pad_to)


def c4_batch(count: int = 256, m_range=(256, 8192)) -> list[Instance]:
    """Batch of independent detectors with uneven M and N (seeded spawn streams)."""
    out = []
    for i in range(count):
        rng = rng_for(4, spawn=i)
        M = int(rng.integers(m_range[0], m_range[1] + 1))
        out.append(random_detector(rng, M, name=f"c4_{i}"))
    return out


def fidelity_columns(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Eq. fidelities for diagonal POVM elements, one value per outcome column:
    (sum_i sqrt(a_i b_i))^2 / (sum_i a_i sum_i b_i) (scoring of a reconstruction against
    a known synthetic POVM; not part of the solver)."""
    num = np.sum(np.sqrt(np.clip(A, 0, None) * np.clip(B, 0, None)), axis=0) ** 2
    den = A.sum(axis=0) * B.sum(axis=0)
    out = np.ones(A.shape[1])
    ok = den > 0
    out[ok] = num[ok] / den[ok]
    return out
