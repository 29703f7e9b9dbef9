"""pdt_smooth_rows_noalloc (the allocation-free smoothing entry point) against
pdt_smooth_rows and the oracle, through the C ABI.

Both entry points run the same kernels in the same order, so their outputs must agree
bit for bit; against the oracle the smoothing tests' bar applies (1e-14 absolute).  Two
calls in a row, the second smaller, check that what the first left in the shared
device array does not leak into the second."""
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


def povm(M, N, seed):
    return simplex.project_rows(np.random.default_rng(seed).normal(size=(M, N)))


def test_two_calls_match_the_allocating_entry_point(dev):
    # the largest first (16384 x 129: 4.2e6 of the 8.4e6 doubles), then a smaller one
    for M, N, divisor, skip, seed in ((16384, 129, 50, 100, 1), (3001, 65, 7, 10, 2)):
        print(f"[noalloc] M={M} N={N} divisor={divisor} skip={skip}", flush=True)
        Pi = povm(M, N, seed)
        x = gpu(Pi, dev)
        want = _pdt.pdt_smooth_rows(x, divisor=divisor, skip=skip)
        got = torch.empty_like(x)
        _pdt.pdt_smooth_rows_noalloc(x, got, divisor=divisor, skip=skip)
        torch.cuda.synchronize()
        assert torch.equal(got, want)
        ref = smoothing.smooth_rows(Pi, divisor, skip)
        assert np.max(np.abs(got.cpu().numpy() - ref)) <= 1e-14


def test_in_place(dev):
    Pi = povm(2000, 9, 3)
    x = gpu(Pi, dev)
    want = _pdt.pdt_smooth_rows(x, divisor=50, skip=100)
    _pdt.pdt_smooth_rows_noalloc(x, x, divisor=50, skip=100)
    torch.cuda.synchronize()
    assert torch.equal(x, want)


def test_sizes_beyond_the_fixed_array_are_rejected(dev):
    # 2 (M + 1 + ceil(M / 256)) N doubles: M = 40000, N = 110 needs 8.8e6 > 8,388,608
    x = torch.zeros((40000, 110), dtype=torch.float64, device=dev)
    with pytest.raises(_pdt.PdtError) as ei:
        _pdt.pdt_smooth_rows_noalloc(x, x)
    assert ei.value.status == _pdt.PDT_ERR_INVALID_ARG
    assert "exceeds" in str(ei.value)
