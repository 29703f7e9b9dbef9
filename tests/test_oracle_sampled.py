"""Pins of the row-at-a-time oracle: on problems small enough to build F, every sampled
row equals the full oracle's row (band membership, residual, gradient, Hessian
diagonal), including the first and last rows, the lumped column and a TRUNCATE case."""
import numpy as np
import pytest

from oracle import fista, objective, poisson, sampled, simplex
from paper_2404_02844_amd import synth


@pytest.mark.parametrize("tail", [synth.LUMP, synth.TRUNCATE])
def test_rows_match_the_full_oracle(tail):
    M = 300
    inst = synth.make_instance("rows", M=M, B=7, eta=0.8, dark=1e-4, D=280, mu_max=(330.0 if tail == synth.LUMP else 250.0),
                               shots=1e6, gamma=2e-3, tail_mode=tail, threshold=1e-16, rng=synth.rng_for(95))
    F, lo, hi = poisson.build_F(inst.mu, M, inst.threshold, tail)
    ro = sampled.RowOracle(inst.mu, M, inst.threshold, tail)
    rng = np.random.default_rng(2)
    Pi = simplex.project_rows(rng.normal(size=(M, inst.N)))
    G = objective.gradient(F, inst.P, Pi, inst.gamma)
    R = objective.residual(F, inst.P, Pi)
    h = fista.hessian_diag(F, inst.gamma, M)
    ms = [0, 1, 2, 57, 150, M - 2, M - 1]
    Fd = F.toarray()
    for m in ms:
        assert ro.probes_of_row(m) == [d for d in range(inst.D) if lo[d] <= m <= hi[d]]
    ds = [0, 1, 100, inst.D - 1]
    assert np.allclose(ro.residual_rows(inst.P, Pi, ds), R[ds], rtol=0, atol=1e-15)
    g = ro.gradient_rows(inst.P, Pi, inst.gamma, ms)
    assert np.max(np.abs(g - G[ms])) <= 1e-13 * np.max(np.abs(G))
    assert np.allclose(ro.hessian_diag_rows(inst.gamma, ms), h[ms], rtol=1e-13, atol=0)
    for d in ds:
        l, v = ro.band(d)
        assert np.array_equal(v, Fd[d, l:l + v.size])


def test_lumped_row_collects_the_high_probes():
    M = 200
    mu = np.linspace(0, 400, 300)
    ro = sampled.RowOracle(mu, M, 1e-16, poisson.LUMP)
    ds = ro.probes_of_row(M - 1)
    # every probe whose tail past M-1 reaches the threshold, up to the last probe
    assert ds[-1] == mu.size - 1
    assert all(poisson.upper_tail(float(mu[d]), M - 1) >= 1e-16 for d in ds)
    assert poisson.upper_tail(float(mu[ds[0] - 1]), M - 1) < 1e-16
