"""Partitioned generation (Sec. 3) through the C ABI against the oracle:
tile counts and every edge of every tile, bit-exact; disjoint row ranges
generated separately add up to the whole graph."""
from __future__ import annotations

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

G500 = (0.57, 0.19, 0.19, 0.05)
CFG3 = (0.45, 0.22, 0.22, 0.11)


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_03525_amd as R
    R.load()
    return R


CASES = [
    # q, k, bound, mode, seed, m, tile_bits, rows
    (G500, 12, 256, oracle.FIXED, 3, 200_000, 3, None),
    (G500, 26, 4096, oracle.VARIABLE, 7, 1 << 22, 6, (5, 9)),
    (CFG3, 34, 1 << 16, oracle.VARIABLE, 3, 1 << 21, 4, None),          # 64-bit ids, L2 table
    (G500, 40, 8192, oracle.VARIABLE, 9, 300_001, 10, (1000, 1024)),    # 64-bit ids, many small tiles
    ((0.25, 0.25, 0.25, 0.25), 16, 1000, oracle.VARIABLE, 1, 100_000, 8, (0, 3)),
    (G500, 2, 100, oracle.VARIABLE, 4, 10_000, 1, None),                 # one letter left per tile
    (G500, 33, 4096, oracle.VARIABLE, 2, 70_000, 1, (1, 2)),
    (G500, 24, 4096, oracle.VARIABLE, 5, 1 << 22, 10, (0, 4)),          # tiles of 1 to 8 blocks packed per wave
]


@pytest.mark.parametrize("q,k,bound,mode,seed,m,tb,rows", CASES)
def test_partition_parity(R, q, k, bound, mode, seed, m, tb, rows):
    r0, r1 = rows if rows else (0, 1 << tb)
    t = R.rmat_build_table(*q, k, bound, mode)
    counts, src, dst = R.generate_partition(t, seed, m, tb, r0, r1)
    o = oracle.build_table(*q, k, bound, mode)
    oc, os_, od = oracle.generate_partition(o, seed, m, tb, r0, r1)
    assert np.array_equal(counts, oc)
    gs, gd = R.to_numpy_ids(src, k), R.to_numpy_ids(dst, k)
    bad = np.nonzero((gs != os_) | (gd != od))[0]
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"
    if rows is None:
        assert int(counts.sum()) == m
    t.close()


def test_row_ranges_add_up_to_the_graph(R):
    """Disjoint row ranges, generated independently, concatenate to the full
    partitioned graph (no communication between the ranges)."""
    import torch
    k, tb, m = 20, 5, 1 << 20
    t = R.rmat_build_table(*G500, k, 4096, R.RMAT_VARIABLE)
    full_c, full_s, full_d = R.generate_partition(t, 13, m, tb)
    parts = [R.generate_partition(t, 13, m, tb, a, b) for a, b in ((0, 7), (7, 8), (8, 32))]
    assert np.array_equal(np.concatenate([p[0] for p in parts]), full_c)
    assert torch.equal(torch.cat([p[1] for p in parts]), full_s)
    assert torch.equal(torch.cat([p[2] for p in parts]), full_d)
    assert int(full_c.sum()) == m
    t.close()


def test_partition_errors(R):
    import torch
    t = R.rmat_build_table(*G500, 16, 256, R.RMAT_VARIABLE)
    x = torch.empty(16, dtype=torch.int32, device="cuda")
    for args in ((100, 0, 0, 1), (100, 16, 0, 1), (100, 3, 4, 4), (100, 3, 0, 9), (2 ** 53 + 1, 3, 0, 1)):
        with pytest.raises(R.RmatError) as ei:
            R.rmat_partition_counts(t, 1, *args)
        assert ei.value.status == R.RMAT_EINVAL
    with pytest.raises(R.RmatError) as ei:      # output size must equal the tiles' edge count
        R.rmat_generate_partition(t, 1, 100, 2, 0, 4, x, x, 16)
    assert ei.value.status == R.RMAT_EINVAL
    t.close()


def test_counts_of_another_table_are_not_reused(R):
    """Counting tiles of one table and then generating those of another
    (same seed, m, tile bits and rows) gives the second table's graph."""
    import torch
    k, tb, m, seed = 20, 4, 200_000, 5
    a = R.rmat_build_table(*G500, k, 4096, R.RMAT_VARIABLE)
    b = R.rmat_build_table(*CFG3, k, 4096, R.RMAT_VARIABLE)
    o = oracle.build_table(*CFG3, k, 4096, oracle.VARIABLE)
    oc, os_, od = oracle.generate_partition(o, seed, m, tb, 0, 1 << tb)
    R.rmat_partition_counts(a, seed, m, tb, 0, 1 << tb)       # a's counts are now the library's last ones
    n = int(oc.sum())
    src = torch.empty(n, dtype=torch.int32, device="cuda")
    dst = torch.empty(n, dtype=torch.int32, device="cuda")
    R.rmat_generate_partition(b, seed, m, tb, 0, 1 << tb, src, dst, n)
    torch.cuda.synchronize()
    assert np.array_equal(R.to_numpy_ids(src, k), os_) and np.array_equal(R.to_numpy_ids(dst, k), od)
    a.close()
    b.close()


def test_async_row_ranges_in_flight_equal_oracle(R):
    """Six row ranges enqueued back to back on one stream by the asynchronous
    entry point (each counted on the host while the previous ones run; six
    calls in flight wrap the ring of four list buffers), synchronised once at
    the end: every range equals the oracle's tiles, and together they hold
    the whole graph."""
    import torch
    k, tb, m, seed = 22, 6, 1 << 22, 11
    t = R.rmat_build_table(*G500, k, 4096, R.RMAT_VARIABLE)
    o = oracle.build_table(*G500, k, 4096, oracle.VARIABLE)
    ranges = [(0, 5), (5, 6), (6, 20), (20, 21), (21, 40), (40, 64)]
    stream = torch.cuda.Stream()
    outs = []
    with torch.cuda.stream(stream):
        for r0, r1 in ranges:
            n = int(R.rmat_partition_counts(t, seed, m, tb, r0, r1).sum())
            src = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
            dst = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
            R.rmat_generate_partition_async(t, seed, m, tb, r0, r1, src, dst, n, stream)
            outs.append((n, src, dst))
    stream.synchronize()
    total = 0
    for (r0, r1), (n, src, dst) in zip(ranges, outs):
        oc, os_, od = oracle.generate_partition(o, seed, m, tb, r0, r1)
        assert int(oc.sum()) == n
        assert np.array_equal(R.to_numpy_ids(src[:n], k), os_), f"rows {r0}..{r1}: src"
        assert np.array_equal(R.to_numpy_ids(dst[:n], k), od), f"rows {r0}..{r1}: dst"
        total += n
    assert total == m
    t.close()


def test_partitioned_workload_full_size_sampled(R):
    """The benchmark's partitioned leg at full size: the k = 26 instance's
    2^30 edges in 256 x 256 tiles, four asynchronous calls of 64 tile rows on
    one stream, each counted on the host before it is enqueued.  Every tile
    count equals the oracle's; the edges of tile rows 1, 63, 64 (the first row
    of the second call), 127, 191 and 255 equal the oracle's tiles."""
    import torch
    import bench
    w = bench.WORKLOAD
    k, m, seed, tb = w["k"], w["m"], w["seed"], 8
    t = R.rmat_build_table(w["a"], w["b"], w["c"], w["d"], k, w["table_bound"], R.RMAT_VARIABLE)
    o = oracle.build_table(w["a"], w["b"], w["c"], w["d"], k, w["table_bound"], oracle.VARIABLE)
    src = torch.empty(m, dtype=torch.int32, device="cuda")
    dst = torch.empty(m, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    counts, n_all = [], 0
    for r0 in range(0, 256, 64):
        c = R.rmat_partition_counts(t, seed, m, tb, r0, r0 + 64)
        n = int(c.sum())
        R.rmat_generate_partition_async(t, seed, m, tb, r0, r0 + 64, src[n_all:], dst[n_all:], n, stream)
        counts.append(c)
        n_all += n
    torch.cuda.synchronize()
    assert n_all == m
    counts = np.concatenate(counts)
    assert np.array_equal(counts, oracle.partition_counts(o, seed, m, tb))
    row_off = np.concatenate([[0], np.cumsum(counts.sum(axis=1))]).astype(np.int64)
    for r in (1, 63, 64, 127, 191, 255):
        _, os_, od = oracle.generate_partition(o, seed, m, tb, r, r + 1)
        a, b = int(row_off[r]), int(row_off[r + 1])
        assert b - a == os_.size
        assert np.array_equal(R.to_numpy_ids(src[a:b], k), os_), f"row {r}: src"
        assert np.array_equal(R.to_numpy_ids(dst[a:b], k), od), f"row {r}: dst"
    del src, dst
    t.close()
