"""Single rows of the problem's quantities, for geometries too large to build F.

Plain definitions restricted to one row at a time, so that a problem with M = 1e6
photon numbers and D = 1e5 probes (a band of ~1e9 entries) can still be checked at
sampled rows:

* ``band``            -- band edges of one probe (the same definition as
                         ``poisson.band_edges``) and its F values;
* ``probes_of_row``   -- the probes whose band holds photon number m;
* ``residual_rows``   -- R_d = sum_m F[d][m] Pi[m] - P_d (Eq. min_obj2);
* ``gradient_rows``   -- grad_m = 2 sum_d F[d][m] R_d + 2 gamma (L Pi)_m;
* ``hessian_diag_rows`` -- h_m = 2 sum_d F[d][m]^2 + 2 gamma L[m][m].

Row membership: for a fixed m, F[d][m] = Poisson(m; mu_d) is unimodal in mu_d (its
derivative in mu has the sign of m - mu), so the probes with F[d][m] >= tau form a
contiguous run of the sorted probe grid around mu = m.  A lumped last column holds
P(X >= M-1; mu), which increases with mu, so its probes form a suffix.  Candidates are
taken from a window around mu = m that is wider than any band, and each is tested with
the probe's exact band edges.
"""
from __future__ import annotations

import math

import numpy as np

from . import poisson


class RowOracle:
    """Caches band edges and F rows of the probes it has touched."""

    def __init__(self, mu: np.ndarray, M: int, tau: float, tail_mode: int):
        self.mu = np.asarray(mu, dtype=np.float64)
        self.M = int(M)
        self.tau = float(tau)
        self.tail_mode = int(tail_mode)
        self._rows: dict[int, tuple[int, np.ndarray]] = {}

    def band(self, d: int) -> tuple[int, np.ndarray]:
        """(lo, F[d][lo..hi]); an empty array when no entry reaches tau."""
        if d not in self._rows:
            lo, hi = poisson.band_edges(float(self.mu[d]), self.M, self.tau, self.tail_mode)
            vals = (poisson.row_values(float(self.mu[d]), lo, hi, self.M, self.tail_mode)
                    if lo <= hi else np.zeros(0))
            self._rows[d] = (lo, vals)
        return self._rows[d]

    def edges(self, d: int) -> tuple[int, int]:
        lo, vals = self.band(d)
        return lo, lo + vals.size - 1

    def probes_of_row(self, m: int) -> list[int]:
        """Probes d with lo_d <= m <= hi_d.

        Inside a probe's band every entry reaches tau except, with a lumped column, the
        stretch between the end of the pmf band and M-1; so a candidate whose entry
        reaches tau is a member, and only candidates below tau whose band may have been
        extended to M-1 have their exact edges computed."""
        M = self.M
        lump = self.tail_mode == poisson.LUMP
        if self.tau <= 0.0:
            return list(range(self.mu.size))
        if lump and m == M - 1:
            a = m - 15.0 * math.sqrt(m + 1.0) - 120.0
            d0 = int(np.searchsorted(self.mu, a, side="left"))
            out = [d for d in range(d0, self.mu.size) if self.edges(d)[1] == M - 1]
            if out and out[0] == d0 and d0 > 0:
                raise RuntimeError("probe window too narrow")
            return out
        a = m - 15.0 * math.sqrt(m + 1.0) - 120.0
        b = m + 15.0 * math.sqrt(m + 15.0 * math.sqrt(m + 1.0) + 240.0) + 240.0
        d0 = int(np.searchsorted(self.mu, a, side="left"))
        d1 = int(np.searchsorted(self.mu, b, side="right"))
        top = M - 1 - 20.0 * math.sqrt(M) - 200.0  # probes whose tail past M-1 may reach tau
        out = []
        for d in range(d0, d1):
            mu_d = float(self.mu[d])
            if float(poisson.pmf(m, mu_d)[0]) >= self.tau:
                out.append(d)
            elif lump and mu_d >= top and mu_d < m:
                lo, hi = self.edges(d)
                if lo <= m <= hi:
                    out.append(d)
        # the window must bracket the run (its ends lie strictly inside it)
        if out and ((out[0] == d0 and d0 > 0) or (out[-1] == d1 - 1 and d1 < self.mu.size)):
            raise RuntimeError("probe window too narrow")
        return out

    def value(self, d: int, m: int) -> float:
        lo, vals = self.band(d)
        k = m - lo
        return float(vals[k]) if 0 <= k < vals.size else 0.0

    def residual_rows(self, P: np.ndarray, Pi: np.ndarray, ds) -> np.ndarray:
        """R_d = F[d] Pi - P_d for each d in ds (FP64 dot products over the band)."""
        N = Pi.shape[1]
        out = np.empty((len(ds), N))
        for k, d in enumerate(ds):
            lo, vals = self.band(d)
            out[k] = (vals @ Pi[lo:lo + vals.size] if vals.size else np.zeros(N)) - P[d]
        return out

    def gradient_rows(self, P: np.ndarray, Pi: np.ndarray, gamma: float, ms) -> np.ndarray:
        """2 sum_d F[d][m] R_d + 2 gamma (L Pi)_m for each m in ms."""
        M, N = Pi.shape
        out = np.empty((len(ms), N))
        for k, m in enumerate(ms):
            ds = self.probes_of_row(m)
            R = self.residual_rows(P, Pi, ds)
            f = np.array([self.value(d, m) for d in ds])
            lap = np.zeros(N)
            if m > 0:
                lap += Pi[m] - Pi[m - 1]
            if m < M - 1:
                lap += Pi[m] - Pi[m + 1]
            for n in range(N):
                out[k, n] = 2.0 * math.fsum(f * R[:, n]) + 2.0 * gamma * lap[n]
        return out

    def hessian_diag_rows(self, gamma: float, ms) -> np.ndarray:
        M = self.M
        out = np.empty(len(ms))
        for k, m in enumerate(ms):
            f = np.array([self.value(d, m) for d in self.probes_of_row(m)])
            ld = 0.0 if M < 2 else (1.0 if m in (0, M - 1) else 2.0)
            out[k] = 2.0 * math.fsum(f * f) + 2.0 * gamma * ld
        return out
