"""The K x K generator cuts a path's base-K value x < 2^15 by K^i with a
multiply-high: floor(x * (floor(2^32 / K^i) + 1) / 2^32).  Exhaustive check
that this equals floor(x / K^i) for every K in 2..16, every K^i in [2, 2^15)
and every x < 2^16 (the kernel needs x < 2^15)."""
from __future__ import annotations

import numpy as np


def test_multiply_high_quotient_is_exact():
    x = np.arange(1 << 16, dtype=np.uint64)
    checked = 0
    for K in range(2, 17):
        d = K
        while d < (1 << 15):
            magic = np.uint64((1 << 32) // d + 1)
            assert int(magic) < (1 << 32)
            q = (x * magic) >> np.uint64(32)
            assert np.array_equal(q, x // np.uint64(d)), (K, d)
            checked += 1
            d *= K
    assert checked > 40
