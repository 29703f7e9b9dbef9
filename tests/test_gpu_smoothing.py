"""Long-range smoothing (Eq. smoothing) on the GPU vs the oracle, through the C ABI.

Tolerance 1e-14 absolute: the kernel forms window sums as differences of compensated
FP64 column prefix sums, accurate to a few ulp of the window sum itself (itself at most
the window's row count, divided by that count in the mean), plus the oracle's own
rounding of a plain sum over up to ~5e4 rows (~1e-15 relative for these values)."""
import numpy as np
import pytest

from oracle import simplex, smoothing
from paper_2404_02844_amd import _pdt

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _pdt.lib()
    return torch.device("cuda:0")


def gpu(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)


@pytest.mark.parametrize("M,N,divisor,skip", [(7, 2, 2, 2), (3000, 9, 50, 100), (4097, 65, 50, 100),
                                              (1000, 130, 7, 0), (300, 1, 3, 10), (50, 5, 50, 100)])
def test_matches_oracle(dev, M, N, divisor, skip):
    print(f"[smooth] M={M} N={N} divisor={divisor} skip={skip}", flush=True)
    Pi = simplex.project_rows(np.random.default_rng(M + N).normal(size=(M, N)))
    out = _pdt.pdt_smooth_rows(gpu(Pi, dev), divisor=divisor, skip=skip).cpu().numpy()
    ref = smoothing.smooth_rows(Pi, divisor, skip)
    assert np.max(np.abs(out - ref)) <= 1e-14
    assert np.array_equal(out[:skip], Pi[:skip])


def test_in_place_and_invariants(dev):
    M, N = 5000, 17
    Pi = simplex.project_rows(np.random.default_rng(4).normal(size=(M, N)))
    t = gpu(Pi, dev)
    _pdt.pdt_smooth_rows(t, out=t)
    out = t.cpu().numpy()
    assert np.max(np.abs(out - smoothing.smooth_rows(Pi))) <= 1e-14
    assert np.all(out >= 0) and np.max(np.abs(out.sum(axis=1) - 1)) <= 1e-14


def test_large_sampled_rows(dev):
    """M = 1.2e6 rows (the paper's experiment has M = 1,210,581), N = 65: sampled rows
    against their window means computed directly."""
    M, N = 1_210_581, 65
    g = torch.Generator(device="cpu").manual_seed(5)
    Pi_h = torch.rand((M, N), generator=g, dtype=torch.float64)
    Pi_h /= Pi_h.sum(dim=1, keepdim=True)
    out = _pdt.pdt_smooth_rows(Pi_h.to(dev)).cpu().numpy()
    P = Pi_h.numpy()
    for i in [0, 99, 100, 101, 4999, 5000, 123457, 600000, 1_000_000, M - 30000, M - 2, M - 1]:
        h = min(i // 50, M - 1 - i)
        ref = P[i - h:i + h + 1].sum(axis=0) / (2 * h + 1) if i >= 100 else P[i]
        assert np.max(np.abs(out[i] - ref)) <= 1e-14, i
