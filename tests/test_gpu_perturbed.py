"""Perturbed-table degree smoothing (Sec. 3) through the C ABI against the
oracle: every member table bit for bit, edge e from member e mod P bit for
bit (with and without the undirected / scramble epilogue), the reduction of
a set, no perturbation equal to the plain table, and the rejected inputs."""
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


def _same_table(g, o):
    assert np.array_equal(g["len"], o.length.astype(np.uint32))
    assert np.array_equal(g["row"], o.row) and np.array_equal(g["col"], o.col)
    assert np.array_equal(g["p"].view(np.uint64), o.p.view(np.uint64))
    assert np.array_equal(g["w"], o.w.astype(np.uint64))
    assert np.array_equal(g["thr"], o.thr) and np.array_equal(g["alias"], o.alias)


SETS = [
    # q, k, bound, mode, P, eps, perturb_seed
    (G500, 20, 4096, oracle.VARIABLE, 4, 0.1, 1),
    (G500, 26, 1024, oracle.VARIABLE, 16, 0.2, 2),
    (CFG3, 34, 256, oracle.FIXED, 8, 0.05, 3),
    (G500, 12, 512, oracle.VARIABLE, 64, 0.5, 4),
    (G500, 30, 8192, oracle.VARIABLE, 8, 0.1, 5),      # 8 x 8192 buckets: set read from global memory
    (G500, 20, 4096, oracle.VARIABLE, 1, 0.3, 6),      # one member
]


@pytest.mark.parametrize("q,k,bound,mode,P,eps,ps", SETS)
def test_member_tables(R, q, k, bound, mode, P, eps, ps):
    t = R.rmat_build_perturbed_table(*q, k, bound, mode, P, eps, ps)
    info = R.rmat_table_info(t)
    assert info["n_tables"] == P
    tabs = oracle.build_perturbed_tables(*q, k, bound, mode, P, eps, ps)
    for i, o in enumerate(tabs):
        _same_table(R.rmat_table_export_member(t, i), o)
    t.close()


EDGES = [
    # set index, seed, edge_begin, m
    (0, 1, 0, 100_000),
    (1, 2, 63, 200_001),
    (2, 3, 2 ** 32 - 5000, 40_000),
    (3, 4, 2 ** 64 - 30_000, 30_000),
    (4, 5, 17, 100_000),
    (5, 6, 5, 10_000),
]


@pytest.mark.parametrize("si,seed,e0,m", EDGES)
def test_set_edge_parity(R, si, seed, e0, m):
    import torch
    q, k, bound, mode, P, eps, ps = SETS[si]
    t = R.rmat_build_perturbed_table(*q, k, bound, mode, P, eps, ps)
    src, dst = R.generate_edges(t, seed, e0, m)
    torch.cuda.synchronize()
    os_, od = oracle.generate_set(oracle.build_perturbed_tables(*q, k, bound, mode, P, eps, ps), seed, e0, m)
    gs, gd = R.to_numpy_ids(src, k), R.to_numpy_ids(dst, k)
    bad = np.nonzero((gs != os_) | (gd != od))[0]
    assert bad.size == 0, f"{bad.size} mismatches, first at {bad[:5]}"
    t.close()


@pytest.mark.parametrize("flags", [1, 2, 3])
def test_set_with_epilogue(R, flags):
    """The epilogue acts on each edge after its member table sampled it:
    edge e equals the oracle's edge e of member e mod P under the same flags."""
    import torch
    q, k, bound, mode, P, eps, ps = SETS[1]
    seed, e0, m, key = 9, 1001, 50_000, 0xC0FFEE
    t = R.rmat_build_perturbed_table(*q, k, bound, mode, P, eps, ps)
    dt = R.id_dtype(k)
    src, dst = torch.empty(m, dtype=dt, device="cuda"), torch.empty(m, dtype=dt, device="cuda")
    R.rmat_generate_ex_async(t, seed, e0, m, flags, key, src, dst)
    torch.cuda.synchronize()
    gs, gd = R.to_numpy_ids(src, k), R.to_numpy_ids(dst, k)
    sel = (np.arange(e0, e0 + m, dtype=np.uint64) % P).astype(np.int64)
    for i, o in enumerate(oracle.build_perturbed_tables(*q, k, bound, mode, P, eps, ps)):
        os_, od = oracle.generate(o, seed, e0, m, threads=8, flags=flags, scramble_key=key)
        mask = sel == i
        assert np.array_equal(gs[mask], os_[mask]) and np.array_equal(gd[mask], od[mask]), f"member {i}"
    t.close()


def test_set_reduction(R):
    """Histogram of src >> (k - b) and XOR of the per-edge mix over a set's
    stream, against the oracle's set stream reduced here."""
    import torch
    q, k, bound, mode, P, eps, ps = SETS[0]
    seed, e0, m, hb = 7, 2 ** 20 - 3, 20_000, 9
    t = R.rmat_build_perturbed_table(*q, k, bound, mode, P, eps, ps)
    hist = torch.zeros(1 << hb, dtype=torch.int64, device="cuda")
    xr = torch.zeros(1, dtype=torch.int64, device="cuda")
    R.rmat_generate_reduce_async(t, seed, e0, m, hb, hist, xr, torch.cuda.current_stream())
    torch.cuda.synchronize()
    os_, od = oracle.generate_set(oracle.build_perturbed_tables(*q, k, bound, mode, P, eps, ps), seed, e0, m)
    oh = np.bincount((os_ >> np.uint32(k - hb)).astype(np.int64), minlength=1 << hb).astype(np.uint64)
    ox = 0
    for j in range(m):
        ox ^= oracle.edge_mix(e0 + j, int(os_[j]), int(od[j]))
    assert np.array_equal(hist.cpu().numpy().view(np.uint64), oh)
    assert int(xr.cpu().numpy().view(np.uint64)[0]) == ox
    t.close()


def test_no_perturbation_is_the_plain_table(R):
    import torch
    a = R.rmat_build_perturbed_table(*G500, 26, 4096, R.RMAT_VARIABLE, 8, 0.0, 77)
    b = R.rmat_build_table(*G500, 26, 4096, R.RMAT_VARIABLE)
    gb = R.rmat_table_export(b)
    for i in range(8):
        ga = R.rmat_table_export_member(a, i)
        for f in gb:
            assert np.array_equal(ga[f], gb[f]), f
    sa, da = R.generate_edges(a, 3, 0, 1 << 20)
    sb, db = R.generate_edges(b, 3, 0, 1 << 20)
    torch.cuda.synchronize()
    assert torch.equal(sa, sb) and torch.equal(da, db)
    a.close()
    b.close()


def test_perturbed_rejections(R):
    for P, eps in ((3, 0.1), (0, 0.1), (128, 0.1), (4, -0.1), (4, 1.0), (4, float("nan"))):
        with pytest.raises(R.RmatError) as ei:
            R.rmat_build_perturbed_table(*G500, 20, 4096, R.RMAT_VARIABLE, P, eps, 1)
        assert ei.value.status == R.RMAT_EINVAL
    t = R.rmat_build_perturbed_table(*G500, 16, 256, R.RMAT_VARIABLE, 4, 0.1, 1)
    with pytest.raises(R.RmatError):
        R.rmat_partition_counts(t, 1, 100, 2)
    for i in (-1, 4):
        with pytest.raises(R.RmatError):
            R.rmat_table_export_member(t, i)
    t.close()
    plain = R.rmat_build_table(*G500, 16, 256, R.RMAT_VARIABLE)
    g = R.rmat_table_export_member(plain, 0)       # a plain table is its own single member
    for f, v in R.rmat_table_export(plain).items():
        assert np.array_equal(g[f], v)
    plain.close()
