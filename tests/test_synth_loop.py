"""The loop-detector generator (Eq. pj_fock and the clicked-bin count) against brute
force: the exact one-bin-at-a-time recursion equals the sum over all 2^J click patterns
of independent bins, and the bin probabilities follow the printed closed forms."""
import itertools

import numpy as np

from paper_2404_02844_amd import synth


def test_bin_probabilities_follow_eq_pj_fock():
    R, el, ed = 0.9, 0.8, 0.5
    q = synth.loop_bin_probs(4, R, el, ed)
    assert np.allclose(q, [R * ed] + [(1 - R) ** 2 / R * (R * el) ** (j - 1) * ed for j in (2, 3, 4)], rtol=1e-15)


def test_poisson_binomial_against_all_click_patterns():
    J, R, el, ed = 6, 0.7, 0.9, 0.5
    q = synth.loop_bin_probs(J, R, el, ed)
    Pi = synth.loop_detector_povm(40, J=J, R=R, eta_loop=el, eta_det=ed, block=7)
    for i in (0, 1, 3, 17, 39):
        p = 1 - (1 - q) ** i
        ref = np.zeros(J + 1)
        for bits in itertools.product([0, 1], repeat=J):
            ref[sum(bits)] += np.prod([p[j] if b else 1 - p[j] for j, b in enumerate(bits)])
        assert np.allclose(Pi[i], ref, rtol=0, atol=1e-15), i
    assert np.allclose(Pi.sum(axis=1), 1.0, atol=1e-15) and np.all(Pi >= 0)


def test_paper_device_occupies_about_fifty_outcomes():
    # the paper's fitted device reaches ~50 outcomes at the top of its Hilbert space
    # (Sec. 2.1: "the first ~50 outcomes are occupied")
    synth._POOL_Q = synth.loop_bin_probs(150, synth.LOOP_R, synth.LOOP_ETA_LOOP, synth.LOOP_ETA_DET)
    try:
        row = synth._loop_rows((1_163_812, 1_163_813))[0]
    finally:
        synth._POOL_Q = None
    occ = np.flatnonzero(row > 1e-6)
    assert abs(row.sum() - 1.0) <= 1e-12
    assert 45 <= occ.max() <= 60 and occ.min() >= 30
