"""Batches through the C ABI: every instance of a batch equals the plain
per-instance path (rmat_build_table + rmat_generate with the same
arguments) and the CPU oracle; graph replays equal the eager run; the
autotuner is deterministic; the 512-instance workload at full size."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1905_03525_amd import workloads

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


def _alloc(R, insts):
    import torch
    for p in insts:
        dt = R.id_dtype(p["k"])
        p["out_src"] = torch.full((p["m"],), -1, dtype=dt, device="cuda")
        p["out_dst"] = torch.full((p["m"],), -1, dtype=dt, device="cuda")
    torch.cuda.synchronize()


def _plain(R, p):
    """Plain path: own table, own launch."""
    import torch
    t = R.rmat_build_table(p["a"], p["b"], p["c"], p["d"], p["k"], p["table_bound"], p["path_mode"])
    s = torch.empty(p["m"], dtype=R.id_dtype(p["k"]), device="cuda")
    d = torch.empty_like(s)
    R.rmat_generate_ex_async(t, p["seed"], p["edge_begin"], p["m"], p.get("gen_flags", 0), p.get("scramble_key", 0),
                             s, d, torch.cuda.current_stream())
    torch.cuda.synchronize()
    return t, s, d


def _mixed():
    """Uneven instances: both id widths, both table residencies, FIXED and
    VARIABLE, unaligned and huge edge_begin, m = 0 and m = 1."""
    q = lambda s: workloads.dirichlet_q(np.random.default_rng(1000 + s))  # noqa: E731
    V, F = oracle.VARIABLE, oracle.FIXED
    rows = [
        # q, k, bound, mode, seed, edge_begin, m
        (G500, 16, 256, F, 1, 0, 1 << 16),
        (G500, 26, 4096, V, 7, 12_345_677, 100_003),
        (CFG3, 34, 1 << 16, V, 3, 2**32 - 3000, 9000),    # 64-bit ids, L2 table, crosses e_hi
        (q(1), 12, 300, V, 11, 5, 40_000),
        (q(2), 40, 8192, V, 12, 10**12 + 1, 30_001),      # 64-bit ids, LDS table
        (q(3), 20, 4**5, F, 13, 0, 0),                    # no edges: table only
        (q(4), 24, 1 << 15, V, 14, 63, 65),               # L2 table, 32-bit ids
        (q(5), 10, 5, V, 15, 0, 1),
        (q(6), 64, 2000, V, 2**64 - 1, 2**64 - 777, 777),  # last edges of the stream
        (q(7), 30, 5000, V, 16, 3, 50_000),
        (q(8), 3, 100, V, 17, 0, 4096),
        (G500, 26, 4096, V, 7, 0, 64 * 2048 * 3 + 5),     # several work items of one instance
    ]
    out = [dict(a=x[0][0], b=x[0][1], c=x[0][2], d=x[0][3], k=x[1], table_bound=x[2], path_mode=x[3], seed=x[4],
                edge_begin=x[5], m=x[6]) for x in rows]
    # Sec. 3 epilogues on some instances
    for i, (fl, key) in {1: (3, 0xBEEF), 2: (2, 7), 3: (1, 0), 8: (3, 2**64 - 1)}.items():
        out[i]["gen_flags"], out[i]["scramble_key"] = fl, key
    return out


@pytest.mark.parametrize("work_blocks", [0, 3, 1])
def test_batch_equals_plain_and_oracle(R, work_blocks):
    import torch
    insts = _mixed()
    _alloc(R, insts)
    with R.rmat_batch_create(insts, work_blocks) as b:
        info = R.rmat_batch_get_info(b)
        # one launch per id width and table residency: 32-bit ids on LDS
        # tables and on an L2 table, 64-bit ids on LDS tables (up to 8192
        # buckets) and on an L2 table
        assert info["n_instances"] == len(insts) and info["n_launches"] == 4
        assert info["total_edges"] == sum(p["m"] for p in insts)
        R.rmat_batch_enqueue(b, torch.cuda.current_stream())
        R.rmat_batch_check(b)
        for i, p in enumerate(insts):
            t, s, d = _plain(R, p)
            assert torch.equal(s, p["out_src"]) and torch.equal(d, p["out_dst"]), f"instance {i} differs from plain"
            gt, bt = R.rmat_table_export(t), R.rmat_batch_table_export(b, i)
            for key in gt:
                assert np.array_equal(gt[key], bt[key]), f"instance {i} table {key}"
            assert R.rmat_batch_table_info(b, i) == R.rmat_table_info(t)
            t.close()
            o = oracle.build_table(p["a"], p["b"], p["c"], p["d"], p["k"], p["table_bound"], p["path_mode"])
            os_, od = oracle.generate(o, p["seed"], p["edge_begin"], p["m"], threads=8, flags=p.get("gen_flags", 0),
                                      scramble_key=p.get("scramble_key", 0))
            assert np.array_equal(R.to_numpy_ids(p["out_src"], p["k"]), os_), f"instance {i} src vs oracle"
            assert np.array_equal(R.to_numpy_ids(p["out_dst"], p["k"]), od), f"instance {i} dst vs oracle"


def test_batch_graph_replays_equal_eager(R):
    import torch
    insts = workloads.batch_instances(40, k_min=8, k_max=16)
    for j, p in enumerate(insts):
        p["table_bound"] = 256 << (j % 6)
    _alloc(R, insts)
    stream = torch.cuda.current_stream()
    with R.rmat_batch_create(insts, 16) as b:
        R.rmat_batch_enqueue(b, stream)
        R.rmat_batch_check(b)
        ref = [(p["out_src"].clone(), p["out_dst"].clone()) for p in insts]
        other = R.rmat_build_table(*G500, 20, 1000, R.RMAT_VARIABLE)
        for rep in range(4):
            for p in insts:   # eager work between replays: clear the outputs, run an unrelated launch
                p["out_src"].fill_(-1)
                p["out_dst"].fill_(-1)
            R.generate_edges(other, rep, 0, 1 << 16)
            torch.cuda.synchronize()
            R.rmat_batch_launch_graph(b, stream)
            R.rmat_batch_check(b)
            for i, p in enumerate(insts):
                assert torch.equal(ref[i][0], p["out_src"]) and torch.equal(ref[i][1], p["out_dst"]), \
                    f"replay {rep}, instance {i}"
        other.close()


def test_autotune_deterministic(R):
    """Without outputs the model alone decides: the same instances get the
    same bounds (LDS and L2 candidates 2^8 .. 2^16), fixed bounds are kept."""
    insts = workloads.batch_instances(64)
    insts[5]["table_bound"] = 777
    a = [dict(p) for p in insts]
    rep1 = R.rmat_batch_autotune(a)
    b = [dict(p) for p in insts]
    rep2 = R.rmat_batch_autotune(b)
    assert [p["table_bound"] for p in a] == [p["table_bound"] for p in b]
    assert a[5]["table_bound"] == 777
    assert all(p["table_bound"] in {1 << e for e in range(8, 17)} for j, p in enumerate(a) if j != 5)
    for rep in (rep1, rep2):
        assert rep["n_tuned"] == 63 and rep["n_candidates"] == 9 and rep["measured"] == 0
        assert 128 <= rep["work_blocks"] <= 8192 and rep["chosen"] == 0
        assert rep["calibration_ns"] > 0 and rep["search_seconds"] > 0 and rep["model_ms"] > 0


def test_autotune_measured_choice(R):
    """With outputs the model's bounds are timed against 4096 and 8192 for
    all; the kept choice is the fastest of the three and the batch built
    with it equals the plain launches."""
    import torch
    insts = workloads.batch_instances(24, k_min=12, k_max=18)
    _alloc(R, insts)
    rep = R.rmat_batch_autotune(insts)
    assert rep["measured"] == 1 and rep["chosen"] in (0, 1, 2)
    t = [rep["tuned_ms"], rep["all_4096_ms"], rep["all_8192_ms"]]
    # the model's bounds are kept unless a single size is faster by more than 1%
    assert all(x > 0 for x in t) and t[rep["chosen"]] <= min(t) / 0.99
    if rep["chosen"] == 1:
        assert all(p["table_bound"] == 4096 for p in insts)
    if rep["chosen"] == 2:
        assert all(p["table_bound"] == 8192 for p in insts)
    with R.rmat_batch_create(insts, rep["work_blocks"]) as b:
        R.rmat_batch_enqueue(b, torch.cuda.current_stream())
        R.rmat_batch_check(b)
        for i, p in enumerate(insts):
            tb, s, d = _plain(R, p)
            assert torch.equal(s, p["out_src"]) and torch.equal(d, p["out_dst"]), f"instance {i}"
            tb.close()


def test_batch_l2_and_lds_groups(R):
    """Instances on 4096-, 8192- and 2^15-bucket tables in one batch: one
    launch per table residency (the two LDS sizes share one), every instance
    equal to its plain launch."""
    import torch
    insts = workloads.batch_instances(12, k_min=12, k_max=20)
    for j, p in enumerate(insts):
        p["table_bound"] = (4096, 8192, 1 << 15)[j % 3]
    _alloc(R, insts)
    with R.rmat_batch_create(insts, 64) as b:
        info = R.rmat_batch_get_info(b)
        assert info["n_launches"] == 2 and info["max_buckets"] == 1 << 15
        R.rmat_batch_enqueue(b, torch.cuda.current_stream())
        R.rmat_batch_check(b)
        for i, p in enumerate(insts):
            tb, s, d = _plain(R, p)
            assert torch.equal(s, p["out_src"]) and torch.equal(d, p["out_dst"]), f"instance {i}"
            tb.close()


def test_batch_workload_512_full(R):
    """The 512-instance workload at full size (about 1.7e10 edges): autotuned
    bounds, one graph launch, every instance equal to its plain launch on the
    device, and oracle samples at both ends and in the middle of each."""
    import torch
    insts = workloads.batch_instances()
    _alloc(R, insts)
    rep = R.rmat_batch_autotune(insts)
    stream = torch.cuda.current_stream()
    m_max = max(p["m"] for p in insts)
    s_all = torch.empty(m_max, dtype=torch.int32, device="cuda")
    d_all = torch.empty(m_max, dtype=torch.int32, device="cuda")
    with R.rmat_batch_create(insts, rep["work_blocks"]) as b:
        R.rmat_batch_launch_graph(b, stream)
        R.rmat_batch_check(b)
        rng = np.random.default_rng(512)
        for i, p in enumerate(insts):
            t = R.rmat_build_table(p["a"], p["b"], p["c"], p["d"], p["k"], p["table_bound"], p["path_mode"])
            s, d = s_all[:p["m"]], d_all[:p["m"]]
            R.rmat_generate_async(t, p["seed"], 0, p["m"], s, d, stream)
            torch.cuda.synchronize()
            assert torch.equal(s, p["out_src"]) and torch.equal(d, p["out_dst"]), f"instance {i} differs from plain"
            t.close()
            o = oracle.build_table(p["a"], p["b"], p["c"], p["d"], p["k"], p["table_bound"], p["path_mode"])
            m = p["m"]
            for e0 in (0, int(rng.integers(0, m - 256)), m - 256):
                os_, od = oracle.generate(o, p["seed"], e0, 256, threads=1)
                gs = R.to_numpy_ids(p["out_src"][e0:e0 + 256], p["k"])
                gd = R.to_numpy_ids(p["out_dst"][e0:e0 + 256], p["k"])
                assert np.array_equal(gs, os_) and np.array_equal(gd, od), f"instance {i} at {e0} vs oracle"
    for p in insts:
        p["out_src"] = p["out_dst"] = None
    torch.cuda.empty_cache()


def test_batch_rejections(R):
    """Inputs refused before any device work: a work list beyond 2^28 items
    (m = 2^60 would otherwise grow it without bound), unknown flags, NULL
    outputs, edge ranges past 2^64; the outputs are never touched."""
    import torch
    buf = torch.full((16,), -1, dtype=torch.int32, device="cuda")
    base = dict(a=G500[0], b=G500[1], c=G500[2], d=G500[3], k=26, table_bound=4096, path_mode=R.RMAT_VARIABLE,
                seed=1, edge_begin=0, m=16, out_src=buf, out_dst=buf)
    for change, status in (({"m": 1 << 60}, R.RMAT_EINVAL), ({"gen_flags": 4}, R.RMAT_EINVAL),
                           ({"out_src": None}, R.RMAT_EINVAL), ({"edge_begin": 2**64 - 8}, R.RMAT_ERANGE)):
        with pytest.raises(R.RmatError) as ei:
            R.rmat_batch_create([dict(base, **change)], 2048)
        assert ei.value.status == status, change
    with pytest.raises(R.RmatError) as ei:
        R.rmat_batch_create([dict(base, m=1 << 60)], 1)
    assert "work items" in str(ei.value)
    torch.cuda.synchronize()
    assert int((buf != -1).sum().item()) == 0


def test_batch_with_failing_build_terminates_and_reports(R):
    """An instance whose parameters admit no fixed-point table (inside the
    validation tolerance, refused by the oracle) is built and generated in
    the same launch as the others: the launch ends, rmat_batch_check reports
    RMAT_EINVAL and names the instance, and the other instances equal their
    plain launches."""
    import torch
    bad = (0.57, 0.19, 0.19, 0.05 - 9e-10)
    insts = [dict(a=G500[0], b=G500[1], c=G500[2], d=G500[3], k=20, table_bound=4096, path_mode=R.RMAT_VARIABLE,
                  seed=5, edge_begin=0, m=1 << 18),
             dict(a=bad[0], b=bad[1], c=bad[2], d=bad[3], k=26, table_bound=5, path_mode=R.RMAT_VARIABLE,
                  seed=6, edge_begin=0, m=1 << 20),
             dict(a=bad[0], b=bad[1], c=bad[2], d=bad[3], k=40, table_bound=5, path_mode=R.RMAT_VARIABLE,
                  seed=7, edge_begin=0, m=1 << 16),
             dict(a=CFG3[0], b=CFG3[1], c=CFG3[2], d=CFG3[3], k=30, table_bound=1 << 15, path_mode=R.RMAT_VARIABLE,
                  seed=8, edge_begin=3, m=100_000)]
    _alloc(R, insts)
    with R.rmat_batch_create(insts, 64) as b:
        R.rmat_batch_enqueue(b, torch.cuda.current_stream())
        torch.cuda.synchronize()
        with pytest.raises(R.RmatError) as ei:
            R.rmat_batch_check(b)
        assert ei.value.status == R.RMAT_EINVAL and "instance 1" in str(ei.value)
        for i in (0, 3):
            p = insts[i]
            t, s, d = _plain(R, p)
            assert torch.equal(s, p["out_src"]) and torch.equal(d, p["out_dst"]), f"instance {i}"
            t.close()
