"""Pins of the long-range smoothing of Eq. smoothing (Sec. 3.2): a hand-computed case,
the averaging matrix built from window membership, and invariants that fix the window
(a symmetric window reproduces linear columns exactly; an off-centre one would not)."""
import numpy as np

from oracle import simplex, smoothing


def test_hand_computed_rows():
    # divisor 2, skip 2, M = 7: half widths 1, 1, 2 (rows 2, 3, 4), then 1 and 0 at the top
    col = np.arange(7, dtype=np.float64) ** 2
    Pi = col[:, None] * np.array([[1.0, -1.0]])
    out = smoothing.smooth_rows(Pi, divisor=2, skip=2)
    exp = np.array([col[0], col[1], (1 + 4 + 9) / 3, (4 + 9 + 16) / 3, (4 + 9 + 16 + 25 + 36) / 5,
                    (16 + 25 + 36) / 3, col[6]])
    assert np.allclose(out[:, 0], exp, rtol=1e-15) and np.allclose(out[:, 1], -exp, rtol=1e-15)


def test_matches_the_window_membership_matrix():
    rng = np.random.default_rng(1)
    M, divisor, skip = 400, 7, 30
    Pi = rng.random((M, 5))
    W = np.zeros((M, M))
    for i in range(M):
        if i < skip:
            W[i, i] = 1.0
            continue
        h = min(i // divisor, M - 1 - i)
        members = [j for j in range(M) if abs(i - j) <= h]
        assert len(members) == 2 * h + 1
        W[i, members] = 1.0 / len(members)
    assert np.allclose(smoothing.smooth_rows(Pi, divisor, skip), W @ Pi, rtol=1e-13, atol=1e-15)


def test_invariants():
    rng = np.random.default_rng(0)
    M = 3000
    Pi = simplex.project_rows(rng.normal(size=(M, 9)))
    out = smoothing.smooth_rows(Pi)
    assert np.array_equal(out[:100], Pi[:100])
    assert np.all(out >= 0) and np.max(np.abs(out.sum(axis=1) - 1)) <= 1e-14
    # constant and linear columns are reproduced (windows are centred on their row)
    i = np.arange(M, dtype=np.float64)
    lin = np.stack([np.full(M, 0.25), 1.0 + 2e-3 * i, 5.0 - 1e-3 * i], axis=1)
    assert np.allclose(smoothing.smooth_rows(lin), lin, rtol=1e-13, atol=0)
    # a divisor beyond M leaves every window at one row
    assert np.array_equal(smoothing.smooth_rows(Pi, divisor=M + 1, skip=0), Pi)
