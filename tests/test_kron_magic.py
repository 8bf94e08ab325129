"""The K x K generator's two integer divisions by a power of K.

64-bit ids cut a path's base-K value x < 2^15 by K^i with a multiply-high:
floor(x * (floor(2^32 / K^i) + 1) / 2^32).  Exhaustive check that this
equals floor(x / K^i) for every K in 2..16, every K^i in [2, 2^15) and every
x < 2^16 (the kernel needs x < 2^15).

32-bit ids append every path whole and divide the value V < 2^47 once by
D = K^d (d digits past k, D <= 2^15; the quotient is an id below 2^32) as
the truncated IEEE double product V * rcp, rcp the double one unit in the
last place above the rounded 1 / D.  Checked for every such D at the
quotients and remainders where rounding could matter (q near 0, 2^31 and
2^32, r = 0, 1, D - 1) and at random ones."""
from __future__ import annotations

from fractions import Fraction

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


def _rcp(d: int) -> np.float64:
    """the double one unit in the last place above the rounded 1 / d"""
    bits = np.array([np.float64(1.0) / np.float64(d)]).view(np.uint64) + np.uint64(1)
    return bits.view(np.float64)[0]


def test_double_quotient_of_the_whole_last_path_is_exact():
    rng = np.random.default_rng(11)
    checked = 0
    for K in range(2, 17):
        for d_exp in range(0, 16):
            D = K ** d_exp
            if D > (1 << 15):
                break
            r = _rcp(D)
            # exactly: 1 / D <= rcp <= (1 / D)(1 + 2^-51)
            assert Fraction(1, D) <= Fraction(float(r)) <= Fraction(1, D) * (1 + Fraction(1, 2 ** 51))
            qs = np.concatenate([np.array([0, 1, 2, (1 << 31) - 1, 1 << 31, (1 << 32) - 2, (1 << 32) - 1],
                                          dtype=np.uint64),
                                 rng.integers(0, 1 << 32, 4000, dtype=np.uint64)])
            rems = np.unique(np.array([0, 1, D - 1, D // 2], dtype=np.uint64))
            rems = rems[rems < np.uint64(D)]
            for rem in np.concatenate([rems, rng.integers(0, D, 8, dtype=np.uint64)]):
                v = qs * np.uint64(D) + np.uint64(rem)
                keep = v < np.uint64(1 << 47)
                vv, qq = v[keep], qs[keep]
                # the kernel forms V as hi * 2^32 + lo in one fused multiply-add (exact below 2^53)
                hi = (vv >> np.uint64(32)).astype(np.float64)
                lo = (vv & np.uint64(0xFFFFFFFF)).astype(np.float64)
                vd = hi * np.float64(4294967296.0) + lo
                assert np.array_equal(vd.astype(np.uint64), vv)
                got = np.trunc(vd * r).astype(np.uint64)
                assert np.array_equal(got, qq), (K, D, int(rem))
            checked += 1
    assert checked > 60
