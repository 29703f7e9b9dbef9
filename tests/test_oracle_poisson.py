"""Pins of the oracle's probe matrix F (Eq. Fmatrix) against 60-digit arithmetic."""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import poisson

mp.mp.dps = 60


def mp_pmf(m, mu):
    if mu == 0:
        return mp.mpf(1) if m == 0 else mp.mpf(0)
    mu = mp.mpf(mu)
    return mp.exp(m * mp.log(mu) - mu - mp.loggamma(m + 1))


def mp_upper_tail(mu, k):
    # P(X >= k) for X ~ Poisson(mu) equals the regularised lower incomplete gamma
    # P(k, mu) = 1 - Q(k, mu); mpmath's upper form converges at mu ~ 1e6 where the lower
    # series does not
    return 1 - mp.gammainc(k, mp.mpf(mu), mp.inf, regularized=True)


@pytest.mark.parametrize("mu", [0.37, 3.0, 40.0, 977.25, 4500.0, 1.1e5, 1e6])
def test_pmf_matches_high_precision(mu):
    sd = math.sqrt(mu)
    ms = sorted({0, 1, 2, int(mu), int(mu) + 1, int(mu + sd), max(0, int(mu - sd)),
                 int(mu + 5 * sd), max(0, int(mu - 5 * sd)), int(mu + 8 * sd), max(0, int(mu - 8 * sd))})
    got = poisson.pmf(np.array(ms), mu)
    for m, g in zip(ms, got):
        ref = mp_pmf(m, mu)
        if ref < mp.mpf("1e-300"):
            assert g < 1e-290
            continue
        rel = abs(mp.mpf(g) - ref) / ref
        # near the mode the saddle-point form is good to a few ulp; in the far tails
        # (entries below 1e-12, where x log(x/mu) and mu - x cancel) to ~1e-13 relative
        tol = 2e-14 if ref > mp.mpf("1e-12") else 3e-13
        assert rel < tol, (mu, m, float(rel))


def test_stirlerr_matches_definition():
    for n in list(range(1, 40)) + [100, 1234, 10**6]:
        ref = mp.loggamma(n + 1) - ((n + mp.mpf("0.5")) * mp.log(n) - n + mp.log(2 * mp.pi) / 2)
        got = poisson.stirlerr(n)[0]
        # n <= 15 subtracts ~30-sized terms (log n! and its Stirling form): a few 1e-15
        # absolute; the series used above 15 is good to rounding
        tol = mp.mpf("5e-15") if n <= 15 else mp.mpf("2e-17") + mp.mpf("1e-15") * abs(ref)
        assert abs(mp.mpf(got) - ref) < tol, n


def test_bd0_matches_definition():
    for x, lam in [(10, 9.5), (1000, 1001.3), (1e6, 1e6 + 17), (5, 50), (300, 12.5), (1e6, 9.1e5)]:
        ref = x * mp.log(mp.mpf(x) / lam) + lam - x
        got = poisson.bd0(x, lam)[0]
        assert abs(mp.mpf(got) - ref) <= mp.mpf("1e-14") * abs(ref) + mp.mpf("1e-300")


def test_special_cases():
    # mu = 0: the vacuum probe puts all mass on m = 0
    v = poisson.pmf(np.arange(5), 0.0)
    assert v[0] == 1.0 and np.all(v[1:] == 0.0)
    # m = 0: exp(-mu)
    for mu in [0.1, 7.0, 700.0]:
        assert poisson.pmf(0, mu)[0] == pytest.approx(math.exp(-mu), rel=1e-15)
    # small mu, small m: the textbook formula is exact enough
    for mu in [0.5, 2.0]:
        for m in range(6):
            assert poisson.pmf(m, mu)[0] == pytest.approx(mu**m * math.exp(-mu) / math.factorial(m), rel=1e-14)


@pytest.mark.parametrize("mu,k", [(3.0, 10), (40.0, 63), (4500.0, 4095), (4000.0, 4095), (3900.0, 4095),
                                  (4095.0, 4095), (1.05e6, 999999), (9.99e5, 999999)])
def test_upper_tail(mu, k):
    ref = mp_upper_tail(mu, k)
    got = poisson.upper_tail(mu, k)
    assert abs(mp.mpf(got) - ref) <= mp.mpf("3e-15") * ref + mp.mpf("1e-300"), (float(ref), got)


def test_lumped_rows_sum_to_one():
    # C2 geometry (M=4096, mu in [0, 4500], tau = 1e-16): every band row sums to 1
    M = 4096
    mus = np.linspace(0, 4500, 5000)[::97]
    for mu in mus:
        lo, hi = poisson.band_edges(float(mu), M, 1e-16, poisson.LUMP)
        s = math.fsum(poisson.row_values(float(mu), lo, hi, M, poisson.LUMP))
        assert abs(s - 1.0) < 1e-13, (mu, s)


def test_truncated_rows_lose_the_tail():
    M = 64
    for mu in [0.0, 5.0, 20.0, 40.0]:
        lo, hi = poisson.band_edges(mu, M, 0.0, poisson.TRUNCATE)
        assert (lo, hi) == (0, M - 1)
        s = math.fsum(poisson.row_values(mu, lo, hi, M, poisson.TRUNCATE))
        ref = 1 - (mp_upper_tail(mu, M) if mu > 0 else 0)
        assert abs(s - float(ref)) < 1e-14


@pytest.mark.parametrize("mu", [0.0, 0.9, 25.0, 1000.0, 4095.5, 4400.0, 2.5e5])
def test_band_edges_bracket_threshold(mu):
    M = 4096 if mu < 1e5 else 300000
    tau = 1e-16
    lo, hi = poisson.band_edges(mu, M, tau, poisson.LUMP)

    def val(m):
        if m == M - 1:
            return mp_upper_tail(mu, M - 1) if mu > 0 else mp.mpf(0)
        return mp_pmf(m, mu)

    assert val(lo) >= tau * (1 - 1e-12)
    assert val(hi) >= tau * (1 - 1e-12)
    if lo > 0:
        assert val(lo - 1) < tau * (1 + 1e-12)
    if hi < M - 1:
        assert val(hi + 1) < tau * (1 + 1e-12)


def test_band_of_a_probe_far_beyond_the_cutoff():
    # mu more than 14 sd above M-1: only the lumped column holds mass (it is ~1)
    M = 1000
    lo, hi = poisson.band_edges(5000.0, M, 1e-16, poisson.LUMP)
    assert (lo, hi) == (M - 1, M - 1)
    assert poisson.upper_tail(5000.0, M - 1) == 1.0
    lo, hi = poisson.band_edges(5000.0, M, 1e-16, poisson.TRUNCATE)
    assert lo > hi
