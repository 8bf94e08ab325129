"""The three Sec. 3 instances the benchmark times, at their full size and in
the launch the benchmark times (one call for all 2^30 edges of the k = 26
instance's seed): the undirected scrambled stream, the set of 8 perturbed
tables of bound 1024 and the 3 x 3 Kronecker initiator at k = 17.  The
output is compared with the oracle on sampled edges: the first, a middle
(unaligned) and the last 2^20 edges, and 256 random 64-edge windows."""
from __future__ import annotations

import numpy as np
import pytest

import bench
import oracle

pytestmark = pytest.mark.gpu

W = bench.WORKLOAD
SLICE = 1 << 20


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_03525_amd as R
    R.load()
    return R


def _windows(m: int):
    rng = np.random.default_rng(2019)
    fixed = [(0, SLICE), (m // 2 + 12_345, SLICE), (m - SLICE, SLICE)]
    starts = rng.integers(0, m - 64, 256)
    return fixed + [(int(s), 64) for s in starts]


def _oracle_stream(which: str, k: int):
    seed = W["seed"]
    if which == "epilogue":
        o = oracle.build_table(W["a"], W["b"], W["c"], W["d"], k, W["table_bound"], oracle.VARIABLE)
        return lambda e0, n: oracle.generate(o, seed, e0, n, threads=8, flags=3, scramble_key=0x5EED)
    if which == "perturbed":
        ts = oracle.build_perturbed_tables(W["a"], W["b"], W["c"], W["d"], k, 1024, oracle.VARIABLE, 8, 0.1, 2019)
        return lambda e0, n: oracle.generate_set(ts, seed, e0, n)
    o = oracle.kron_build_table(bench.P3, 3, k, 4096, oracle.VARIABLE)
    return lambda e0, n: oracle.generate(o, seed, e0, n, threads=8)


@pytest.mark.parametrize("which", ["epilogue", "perturbed", "kron3x3"])
def test_sec3_workload_full_size_sampled(R, which):
    import torch
    m = W["m"]
    k = 17 if which == "kron3x3" else W["k"]
    t = bench.sec3_tables(R, W["k"])[which]()
    assert R.rmat_table_info(t)["k"] == k
    src = torch.empty(m, dtype=torch.int32, device="cuda")
    dst = torch.empty(m, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    bench.sec3_launch(R, which, t, src, dst, stream)()
    torch.cuda.synchronize()
    ref = _oracle_stream(which, k)
    for e0, n in _windows(m):
        gs = R.to_numpy_ids(src[e0:e0 + n], k)
        gd = R.to_numpy_ids(dst[e0:e0 + n], k)
        os_, od = ref(e0, n)
        bad = np.nonzero((gs != os_) | (gd != od))[0]
        assert bad.size == 0, f"{which}: {bad.size} mismatches in [{e0}, {e0 + n}), first at {e0 + bad[:5]}"
    del src, dst
    t.close()
