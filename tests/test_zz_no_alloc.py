"""The allocation-free reduction (rmat_generate_reduce_noalloc_async)
through the C ABI: two calls in a row, the second on a smaller input, each
equal to rmat_generate_reduce_async with the same arguments (histogram and
checksum bit for bit), the small one also equal to the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_03525_amd as R
    R.load()
    return R


def _reduce(R, fn, t, seed, e0, m, hb):
    import torch
    hist = torch.zeros(1 << hb, dtype=torch.int64, device="cuda")
    xr = torch.zeros(1, dtype=torch.int64, device="cuda")
    fn(t, seed, e0, m, hb, hist, xr, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return hist.cpu().numpy().view(np.uint64), int(xr.item()) & (2**64 - 1)


def test_noalloc_reduce_equals_allocating_reduce(R):
    cases = [
        # q, k, bound, seed, edge_begin, m, hist_bits: several 2^23-edge sub-chunks and a ragged
        # tail on an L2 table with 64-bit ids, across e = 2^32; then a smaller input on an LDS table
        ((0.45, 0.22, 0.22, 0.11), 34, 1 << 16, 3, 2**32 - 1000, 3 * (1 << 23) + 12_345, 16),
        ((0.57, 0.19, 0.19, 0.05), 26, 4096, 7, 77, 100_003, 11),
    ]
    for q, k, bound, seed, e0, m, hb in cases:
        print(f"noalloc reduce k={k} bound={bound} m={m} hist_bits={hb}", flush=True)
        t = R.rmat_build_table(*q, k, bound, R.RMAT_VARIABLE)
        h_s, x_s = _reduce(R, R.rmat_generate_reduce_noalloc_async, t, seed, e0, m, hb)
        h_a, x_a = _reduce(R, R.rmat_generate_reduce_async, t, seed, e0, m, hb)
        assert int(h_s.sum()) == m
        assert np.array_equal(h_s, h_a) and x_s == x_a, f"k={k}: no-alloc reduction differs"
        if m <= 1 << 20:
            o = oracle.build_table(*q, k, bound, oracle.VARIABLE)
            oh, ox = oracle.generate_reduce(o, seed, e0, m, hb, threads=8)
            assert np.array_equal(h_s, oh) and x_s == ox, f"k={k}: no-alloc reduction vs oracle"
        t.close()


def test_noalloc_reduce_errors(R):
    import torch
    t = R.rmat_build_table(0.57, 0.19, 0.19, 0.05, 12, 256, R.RMAT_VARIABLE)
    hist = torch.zeros(1 << 12, dtype=torch.int64, device="cuda")
    xr = torch.zeros(1, dtype=torch.int64, device="cuda")
    for hb in (-1, 13):
        with pytest.raises(R.RmatError) as ei:
            R.rmat_generate_reduce_noalloc_async(t, 1, 0, 100, hb, hist, xr)
        assert ei.value.status == R.RMAT_EINVAL
    with pytest.raises(R.RmatError) as ei:
        R.rmat_generate_reduce_noalloc_async(t, 1, 2**64 - 10, 20, 4, hist, xr)
    assert ei.value.status == R.RMAT_ERANGE
    R.rmat_generate_reduce_noalloc_async(t, 1, 0, 0, 4, hist, xr)  # m = 0: nothing to do
    torch.cuda.synchronize()
    assert int(hist.sum().item()) == 0 and int(xr.item()) == 0
    t.close()
