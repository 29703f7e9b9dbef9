"""Long-range smoothing of a reconstructed POVM before a second, stage-2-only run
(Sec. 3.2, Eq. smoothing).

Each row i at or above the excluded range is replaced by the mean of the rows within a
photon-number distance N_smooth(i) of it; the paper uses N_smooth(i) = i/50 and leaves
the lowest ~100 photon numbers unchanged.

Readings where the paper is silent (also listed in the design notes):
  * N_smooth(i) = floor(i / divisor) (divisor 50);
  * rows i < skip (100) are copied unchanged;
  * near the top of the photon-number range the window shrinks symmetrically,
    N_eff(i) = min(N_smooth(i), M - 1 - i), so that it stays centred on i and the
    divisor 2 N_eff + 1 of Eq. smoothing counts exactly the rows summed.
Every smoothed row is a mean of rows on the simplex, so it stays on the simplex.
"""
from __future__ import annotations

import numpy as np


def half_width(i: int, M: int, divisor: int) -> int:
    return min(i // divisor, M - 1 - i)


def smooth_rows(Pi: np.ndarray, divisor: int = 50, skip: int = 100) -> np.ndarray:
    """Eq. smoothing row by row: a plain mean over each window, in FP64."""
    M = Pi.shape[0]
    out = np.array(Pi, dtype=np.float64, copy=True)
    for i in range(min(skip, M), M):
        h = half_width(i, M, divisor)
        out[i] = Pi[i - h:i + h + 1].sum(axis=0) / (2 * h + 1)
    return out
