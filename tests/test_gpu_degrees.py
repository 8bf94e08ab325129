"""Out-degree counters and degree distribution through the C ABI against the
oracle: every counter of the graph bit for bit (LDS and L2 tables, fixed and
variable paths, perturbed sets, unaligned edge ranges, calls that accumulate),
64-bit ids on the nodes the edges touch plus the total, the distribution with
and without clipping, a 2^30-edge graph by its sums and against the on-device
source-prefix histogram, and the rejected inputs."""
from __future__ import annotations

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

G500 = (0.57, 0.19, 0.19, 0.05)
SKEW = (0.5, 0.3, 0.1, 0.1)


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_03525_amd as R
    R.load()
    return R


def _degrees(R, t, k, seed, e0, m, parts=1):
    import torch
    deg = torch.zeros(1 << k, dtype=torch.int32, device="cuda")
    step = (m + parts - 1) // parts
    for off in range(0, m, step):
        R.rmat_generate_degrees_async(t, seed, e0 + off, min(step, m - off), deg, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return deg


CASES = [
    # q, k, bound, mode, seed, edge_begin, m, parts
    (G500, 16, 4096, oracle.VARIABLE, 1, 0, 1 << 20, 1),
    (SKEW, 20, 256, oracle.FIXED, 2, 12345, (1 << 21) + 17, 3),
    (G500, 22, 1 << 16, oracle.VARIABLE, 3, 2 ** 33 - 777, 1 << 20, 1),   # L2 table
    ((0.25, 0.25, 0.25, 0.25), 12, 1000, oracle.VARIABLE, 4, 63, 100_001, 2),
    (G500, 1, 100, oracle.VARIABLE, 5, 0, 5000, 1),
    (G500, 20, 16, oracle.VARIABLE, 6, 3, 200_000, 2),   # most edges need a second counter block
]


@pytest.mark.parametrize("q,k,bound,mode,seed,e0,m,parts", CASES)
def test_degrees_equal_oracle(R, q, k, bound, mode, seed, e0, m, parts):
    t = R.rmat_build_table(*q, k, bound, mode)
    deg = _degrees(R, t, k, seed, e0, m, parts).cpu().numpy().view(np.uint32)
    want = oracle.out_degrees(oracle.build_table(*q, k, bound, mode), seed, e0, m)
    assert np.array_equal(deg.astype(np.uint64), want)
    t.close()


def test_perturbed_set_degrees(R):
    q, k, bound, P, eps, ps, seed, e0, m = G500, 18, 1024, 4, 0.2, 7, 9, 5, 300_000
    t = R.rmat_build_perturbed_table(*q, k, bound, R.RMAT_VARIABLE, P, eps, ps)
    deg = _degrees(R, t, k, seed, e0, m).cpu().numpy().view(np.uint32)
    src, _ = oracle.generate_set(oracle.build_perturbed_tables(*q, k, bound, oracle.VARIABLE, P, eps, ps), seed, e0, m)
    assert np.array_equal(deg, np.bincount(src, minlength=1 << k).astype(np.uint32))
    t.close()


def test_wide_ids_touched_nodes(R):
    """k = 33: 2^33 counters (32 GiB); the nodes the oracle's edges touch hold
    their counts and the counters sum to m."""
    import torch
    q, k, bound, seed, e0, m = G500, 33, 4096, 6, 1 << 40, 1 << 20
    t = R.rmat_build_table(*q, k, bound, R.RMAT_VARIABLE)
    deg = _degrees(R, t, k, seed, e0, m)
    src, _ = oracle.generate(oracle.build_table(*q, k, bound, oracle.VARIABLE), seed, e0, m, threads=8)
    nodes, counts = np.unique(src, return_counts=True)
    got = deg[torch.from_numpy(nodes.astype(np.int64)).cuda()].cpu().numpy().view(np.uint32)
    assert np.array_equal(got, counts.astype(np.uint32))
    assert int(deg.sum(dtype=torch.int64).item()) == m
    del deg
    torch.cuda.empty_cache()
    t.close()


@pytest.mark.parametrize("n_cut,max_degree", [(0, 1000), (3, 8), (1, 3), (2, 0)])
def test_distribution_equals_oracle(R, n_cut, max_degree):
    import torch
    q, k, seed, m = G500, 16, 8, 1 << 21
    t = R.rmat_build_table(*q, k, 4096, R.RMAT_VARIABLE)
    deg = _degrees(R, t, k, seed, 0, m)
    n = (1 << k) - n_cut            # counts not a multiple of 4: the tail path
    hist = torch.zeros(max_degree + 1, dtype=torch.int64, device="cuda")
    R.rmat_degree_distribution_async(deg, n, max_degree, hist, torch.cuda.current_stream())
    torch.cuda.synchronize()
    want = oracle.degree_distribution(deg.cpu().numpy().view(np.uint32)[:n].astype(np.uint64), max_degree)
    assert np.array_equal(hist.cpu().numpy().view(np.uint64), want)
    t.close()


def test_large_graph_sums_and_prefix_histogram(R):
    """k = 30, 2^30 edges: the distribution counts 2^30 nodes and 2^30 edges,
    and the counters summed over each 2^14-node source prefix equal the
    on-device prefix histogram of the same edges (itself checked against the
    oracle chunk by chunk)."""
    import torch
    q, k, seed, m = G500, 30, 7, 1 << 30
    t = R.rmat_build_table(*q, k, 4096, R.RMAT_VARIABLE)
    deg = _degrees(R, t, k, seed, 0, m)
    max_degree = 1 << 20
    hist = torch.zeros(max_degree + 1, dtype=torch.int64, device="cuda")
    R.rmat_degree_distribution_async(deg, 1 << k, max_degree, hist, torch.cuda.current_stream())
    torch.cuda.synchronize()
    h = hist.cpu().numpy().view(np.uint64)
    assert int(h.sum()) == 1 << k
    assert int(h[-1]) == 0 and int((np.arange(max_degree + 1, dtype=np.uint64) * h).sum()) == m
    pref = torch.zeros(1 << 16, dtype=torch.int64, device="cuda")
    xr = torch.zeros(1, dtype=torch.int64, device="cuda")
    R.rmat_generate_reduce_async(t, seed, 0, m, 16, pref, xr, torch.cuda.current_stream())
    by_prefix = deg.view(1 << 16, 1 << (k - 16)).sum(dim=1, dtype=torch.int64)
    torch.cuda.synchronize()
    assert torch.equal(by_prefix, pref)
    del deg
    torch.cuda.empty_cache()
    t.close()


def test_degree_rejections(R):
    import torch
    t = R.rmat_build_table(*G500, 12, 256, R.RMAT_VARIABLE)
    deg = torch.zeros(1 << 12, dtype=torch.int32, device="cuda")
    with pytest.raises(R.RmatError):
        R.rmat_generate_degrees_async(t, 1, 0, 10, None)
    with pytest.raises(R.RmatError):
        R.rmat_generate_degrees_async(t, 1, 0, 10, deg.data_ptr() + 2)
    with pytest.raises(R.RmatError) as ei:
        R.rmat_generate_degrees_async(t, 1, 2 ** 64 - 5, 10, deg)
    assert ei.value.status == R.RMAT_ERANGE
    R.rmat_generate_degrees_async(t, 1, 0, 0, None)   # m = 0: nothing to do
    kt = R.rmat_kron_build_table([1 / 9] * 9, 3, 7, 256, R.RMAT_VARIABLE)
    with pytest.raises(R.RmatError):
        R.rmat_generate_degrees_async(kt, 1, 0, 10, deg)
    hist = torch.zeros(9, dtype=torch.int64, device="cuda")
    for args in ((deg, 1 << 12, 8, None), (None, 1 << 12, 8, hist), (deg.data_ptr() + 4, 100, 8, hist),
                 (deg, 1 << 41, 8, hist), (deg, 100, 1 << 31, hist)):
        with pytest.raises(R.RmatError):
            R.rmat_degree_distribution_async(*args)
    torch.cuda.synchronize()
    assert int(deg.sum().item()) == 0 and int(hist.sum().item()) == 0
    kt.close()
    t.close()
