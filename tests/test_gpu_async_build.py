"""rmat_build_table_async: the same table and the same edges as the
synchronous build, with generation ordered after the build on the device
(another stream, no host wait), and a failed build reported later."""
from __future__ import annotations

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

G500 = (0.57, 0.19, 0.19, 0.05)
CFG3 = (0.45, 0.22, 0.22, 0.11)
# inside the 1e-9 sum tolerance, with a largest-remainder residual out of
# range at bound 5: the device build fails
FAILING = (0.57, 0.19, 0.19, 0.05 - 9e-10)


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_03525_amd as R
    R.load()
    return R


def _gen(R, t, k, seed, e0, m, stream):
    import torch
    src = torch.empty(m, dtype=R.id_dtype(k), device="cuda")
    dst = torch.empty_like(src)
    R.rmat_generate_async(t, seed, e0, m, src, dst, stream)
    return src, dst


CASES = [
    # q, k, bound, mode, seed, edge_begin, m
    (G500, 26, 4096, oracle.VARIABLE, 7, 3, 300_001),
    (G500, 26, 16, oracle.VARIABLE, 22, 5, 70_000),       # most edges need two counter blocks
    (CFG3, 34, 1 << 16, oracle.VARIABLE, 3, 2**32 - 3000, 9000),  # L2 table, 64-bit ids
]


@pytest.mark.parametrize("q,k,bound,mode,seed,e0,m", CASES)
def test_async_build_equals_sync(R, q, k, bound, mode, seed, e0, m):
    import torch
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    ts = R.rmat_build_table(*q, k, bound, mode)
    s1, d1 = _gen(R, ts, k, seed, e0, m, main)
    # built on a side stream, generated at once on the main stream: the
    # library orders the generation after the build on the device
    ta = R.rmat_build_table_async(*q, k, bound, mode, side)
    s2, d2 = _gen(R, ta, k, seed, e0, m, main)
    torch.cuda.synchronize()
    assert torch.equal(s1, s2) and torch.equal(d1, d2)
    ia, is_ = R.rmat_table_info(ta), R.rmat_table_info(ts)
    assert ia["device_bytes"] > is_["device_bytes"]  # the build's working arrays stay with the table
    ia.pop("device_bytes"), is_.pop("device_bytes")
    assert ia == is_
    ea, es = R.rmat_table_export(ta), R.rmat_table_export(ts)
    for key in es:
        assert np.array_equal(ea[key], es[key]), key
    # after the build is known to be done (two blocks where the table wants
    # them): the same edges again
    s3, d3 = _gen(R, ta, k, seed, e0, m, side)
    torch.cuda.synchronize()
    assert torch.equal(s1, s3) and torch.equal(d1, d3)
    o = oracle.build_table(*q, k, bound, mode)
    os_, od = oracle.generate(o, seed, e0, min(m, 20_000), threads=8)
    assert np.array_equal(R.to_numpy_ids(s2, k)[:len(os_)], os_)
    assert np.array_equal(R.to_numpy_ids(d2, k)[:len(od)], od)
    ta.close()
    ts.close()


def test_async_builds_back_to_back_on_one_stream(R):
    """Build, generate, build, generate on one stream with no host wait: each
    generation uses its own table."""
    import torch
    s = torch.cuda.current_stream()
    outs = []
    tables = []
    for seed, bound in ((1, 4096), (2, 256), (3, 1000)):
        t = R.rmat_build_table_async(*G500, 20, bound, R.RMAT_VARIABLE, s)
        tables.append(t)
        outs.append(_gen(R, t, 20, seed, 0, 50_000, s))
    torch.cuda.synchronize()
    for (seed, bound), (src, dst), t in zip(((1, 4096), (2, 256), (3, 1000)), outs, tables):
        ref = R.rmat_build_table(*G500, 20, bound, R.RMAT_VARIABLE)
        s2, d2 = _gen(R, ref, 20, seed, 0, 50_000, s)
        torch.cuda.synchronize()
        assert torch.equal(src, s2) and torch.equal(dst, d2)
        ref.close()
        t.close()


def test_failed_async_build_is_reported(R):
    import torch
    with pytest.raises(R.RmatError) as sync_err:
        R.rmat_build_table(*FAILING, 26, 5, R.RMAT_VARIABLE)
    assert sync_err.value.status == R.RMAT_EINVAL
    s = torch.cuda.current_stream()
    t = R.rmat_build_table_async(*FAILING, 26, 5, R.RMAT_VARIABLE, s)  # sizing passes; the device build fails
    # a generation launched before the failure is known ends (terminating records)
    _gen(R, t, 26, 1, 0, 100_000, s)
    torch.cuda.synchronize()
    with pytest.raises(R.RmatError) as e:
        R.rmat_table_info(t)
    assert e.value.status == R.RMAT_EINVAL
    with pytest.raises(R.RmatError) as e2:
        _gen(R, t, 26, 1, 0, 1000, s)
    assert e2.value.status == R.RMAT_EINVAL
    t.close()
