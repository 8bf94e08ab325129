"""Benchmark of the R-MAT sampler on one MI355X.

A step is one pass of the whole hot path over the benchmark instance: build
the 4096-entry variable-length path table for a=0.57, b=c=0.19, d=0.05,
k=26 (validation, path enumeration, quantisation, alias table, bucket
records), then generate m = 16 * 2^26 = 2^30 edges (Philox draws, alias
lookups, concatenation, stores of uint32 source and destination ids) into
device memory.  One JSON line is printed.  Beside it: the 512-instance
batched workload as one hipGraph launch against 512 plain launches
(`batched_speedup`), a window of the served request stream against plain
per-request launches (`served`), the k=34 instance in 2^30-edge chunks
reduced on the device (`k34`), and the CPU oracle on a bounded sample
(`cpu_baseline`).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-batch]
                    [--served-window S] [--served-reading A|B] [--served-pool P]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = dict(name="rmat_k26_ef16_var4096", a=0.57, b=0.19, c=0.19, d=0.05, k=26, m=1 << 30,
                table_bound=4096, path_mode="variable", seed=7)
HBM_PEAK_GBS = 8000.0
BYTES_PER_EDGE = 8  # two uint32 ids written per edge
# integer VALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one 32-bit op per lane per cycle)
PEAK_CLOCK_GHZ = 2.4
INT_PEAK_OPS = 256 * 4 * 16 * PEAK_CLOCK_GHZ * 1e9
OPS_PER_PHILOX_BLOCK = 40  # 20 products 32x32->64 + 20 three-input XORs (10 rounds)
OPS_PER_SAMPLE = 11        # shift, compare, 2 selects, row/col split (2), 2 shifts, 2 ORs, add
OPS_EPILOGUE = 21          # mirror (compare + 2 selects) + per id 3 rounds of (multiply-add, field extract, and-xor)
OPS_KRON_CUT = 2           # K x K: the last path's two digit values divided by K^i (one multiply-high each)
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "generate_k26_ef16_traffic.txt")
POWER_CLOCK_SUMMARY = os.path.join(ROOT, "profiles", "generate_k26_ef16_power_clock.txt")


def samples_per_edge(table_export: dict, k: int):
    """E[N] and E[ceil(N/4)] for N = samples until k letters, from the
    table's own weights and path lengths (renewal recursion over the letter
    count)."""
    import numpy as np
    w = table_export["w"].astype(np.float64) / 2.0**32
    L = table_export["len"].astype(np.int64)
    pl = np.bincount(L[w > 0], weights=w[w > 0], minlength=16)
    state = np.zeros(k)
    state[0] = 1.0
    en, eb = 0.0, 0.0
    for n in range(1, 4 * k + 8):
        nxt = np.zeros(k)
        done = 0.0
        for f in np.nonzero(state)[0]:
            for length in np.nonzero(pl)[0]:
                if f + length >= k:
                    done += state[f] * pl[length]
                else:
                    nxt[f + length] += state[f] * pl[length]
        en += n * done
        eb += ((n + 3) // 4) * done
        state = nxt
    return en, eb


def alu_roofline(kernel_ms: float, m: int, ops_per_edge: float) -> dict:
    """Integer-ALU roofline of one generation kernel: algorithmic ops per edge
    times the edges of the launch over its duration, against the VALU peak."""
    achieved = ops_per_edge * m / (kernel_ms / 1e3)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": INT_PEAK_OPS / 1e12, "unit": "Tops/s",
            "frac": achieved / INT_PEAK_OPS, "ops_per_edge": ops_per_edge}


def _cpu_model() -> str:
    """The host CPU as /proc/cpuinfo names it, with family / model / stepping
    (a virtual machine may report only a short model name) and whether it
    runs under a hypervisor."""
    fields = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if not line.strip():
                    break  # the first processor's block is enough
                key, _, val = line.partition(":")
                fields[key.strip()] = val.strip()
    except OSError:
        return "unknown"
    name = fields.get("model name", "unknown")
    extra = [f"{k} {fields[k]}" for k in ("cpu family", "model", "stepping") if k in fields]
    if "hypervisor" in fields.get("flags", "").split():
        extra.append("under a hypervisor")
    return name + (" (" + ", ".join(extra) + ")" if extra else "")


def _host_cpus() -> dict:
    """CPUs of this host: os.cpu_count(), the ones this process may run on
    (affinity), and the cgroup CPU quota if one is set."""
    out = {"cpu_count": os.cpu_count() or 1}
    try:
        out["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        out["affinity"] = out["cpu_count"]
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            quota, period = f.read().split()[:2]
        if quota != "max":
            out["cgroup_quota"] = int(quota) / int(period)
    except (OSError, ValueError):
        pass
    return out


def cpu_baseline(budget_s: float = 12.0) -> dict:
    """The oracle as it stands, on every CPU this process may use (affinity,
    capped by a cgroup quota), over the edges of the same instance in
    2^24-edge slices from edge 0 until the whole instance is done or the
    time budget is used; one 2^22-edge slice on one thread beside it."""
    import oracle
    host = _host_cpus()
    threads = host["affinity"]
    if "cgroup_quota" in host:
        threads = max(1, min(threads, int(host["cgroup_quota"])))
    w = WORKLOAD
    t = oracle.build_table(w["a"], w["b"], w["c"], w["d"], w["k"], w["table_bound"], oracle.VARIABLE)
    sl = 1 << 24
    done, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s and done < w["m"]:
        oracle.generate(t, w["seed"], done, sl, threads=threads)
        done += sl
    el = time.perf_counter() - t0
    t1 = time.perf_counter()
    oracle.generate(t, w["seed"], 0, 1 << 22, threads=1)
    one = (1 << 22) / (time.perf_counter() - t1)
    whole = " (the whole instance)" if done >= w["m"] else ""
    return {"value": done / el, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": f"edges [0, {done}){whole} of the same instance in 2^24-edge slices, {el:.1f} s",
            "one_thread_value": one, "cpu_model": _cpu_model(), "host_cpus": host}


def batched_vs_plain(R, reps: int = 3) -> dict:
    """The 512-instance workload: one hipGraph launch of the batch (all 512
    table builds and every instance's edges) against 512 plain
    rmat_build_table_async + rmat_generate_async calls on one stream, both timed by
    the host clock from the first call to the final synchronisation.  The
    autotuned bounds are also compared, as graph launches, with 4096 and
    with 8192 for every instance."""
    import torch
    from paper_1905_03525_amd import workloads
    insts = workloads.batch_instances()
    for p in insts:
        p["out_src"] = torch.empty(p["m"], dtype=torch.int32, device="cuda")
        p["out_dst"] = torch.empty(p["m"], dtype=torch.int32, device="cuda")
    rep = R.rmat_batch_autotune(insts)
    total = sum(p["m"] for p in insts)
    stream = torch.cuda.current_stream()

    def plain():
        tables = []
        for p in insts:
            t = R.rmat_build_table_async(p["a"], p["b"], p["c"], p["d"], p["k"], p["table_bound"], p["path_mode"],
                                         stream)
            R.rmat_generate_async(t, p["seed"], 0, p["m"], p["out_src"], p["out_dst"], stream)
            tables.append(t)
        torch.cuda.synchronize()
        for t in tables:
            t.close()

    def graph_ms(bounds, work_blocks):
        """median host-clock ms of `reps` graph launches of the batch with
        these bounds (after the capture run)"""
        trial = [dict(p, table_bound=bd) for p, bd in zip(insts, bounds)]
        b = R.rmat_batch_create(trial, work_blocks)
        R.rmat_batch_launch_graph(b, stream)   # capture + warm-up
        R.rmat_batch_check(b)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            R.rmat_batch_launch_graph(b, stream)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        R.rmat_batch_check(b)
        info = R.rmat_batch_get_info(b)
        b.close()
        return sorted(ts)[len(ts) // 2] * 1e3, info

    tuned = [p["table_bound"] for p in insts]
    fixed_4096, _ = graph_ms([4096] * len(insts), rep["work_blocks"])
    fixed_8192, _ = graph_ms([8192] * len(insts), rep["work_blocks"])
    b = R.rmat_batch_create(insts, rep["work_blocks"])
    info = R.rmat_batch_get_info(b)
    R.rmat_batch_launch_graph(b, stream)   # capture + warm-up
    R.rmat_batch_check(b)
    plain()                                # warm-up
    t_graph, t_plain = [], []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        R.rmat_batch_launch_graph(b, stream)
        torch.cuda.synchronize()
        t_graph.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        plain()
        t_plain.append(time.perf_counter() - t0)
    R.rmat_batch_check(b)
    b.close()
    for p in insts:
        p["out_src"] = p["out_dst"] = None
    torch.cuda.empty_cache()
    tg, tp = sorted(t_graph)[len(t_graph) // 2], sorted(t_plain)[len(t_plain) // 2]
    return {"workload": "batch512_k10-24_ef4-32_dirichlet4221", "instances": len(insts), "total_edges": total,
            "graph_ms": tg * 1e3, "plain_ms": tp * 1e3, "speedup": tp / tg, "graph_edges_per_s": total / tg,
            "plain_edges_per_s": total / tp, "autotune_search_s": rep["search_seconds"],
            "autotune_choice": ["model", "all_4096", "all_8192"][rep["chosen"]],
            "autotune_timed_ms": {"model": rep["tuned_ms"], "all_4096": rep["all_4096_ms"],
                                  "all_8192": rep["all_8192_ms"]},
            "autotune_model_ms": rep["model_ms"],
            "autotune_calibration_ns_per_edge_op": rep["calibration_ns"], "work_blocks": rep["work_blocks"],
            "graph_ms_all_4096": fixed_4096, "graph_ms_all_8192": fixed_8192,
            "n_work_items": info["n_work_items"], "n_launches": info["n_launches"], "tile_blocks": info["tile_blocks"],
            "bounds_histogram": {str(v): tuned.count(v) for v in sorted(set(tuned))}}


def served_vs_plain(R, window_s: float, reading: str = "A", rate: float = 2000.0, plain: bool = True,
                    pool: int = 0) -> dict:
    """The served workload: a Poisson stream of R-MAT requests (k per
    `reading`, edge factor 8 or 16, Dirichlet(4,2,2,1) parameters, table bound
    4096) at `rate` requests/s; the first `window_s` seconds of arrivals go
    through the request server (200 GB output arena, device table cache,
    continuous batching), outputs released as each request completes.  The
    same requests are then generated one after another by plain
    rmat_build_table_async + rmat_generate_async calls.  pool > 0: parameters from
    that many pre-drawn sets, so the table cache can hit."""
    import torch
    from paper_1905_03525_amd import workloads
    reqs = workloads.served_requests(rate=rate, duration=window_s, arrival_seed=2019, reading=reading, pool=pool)
    for p in reqs:
        p["flags"] = R.RMAT_REQ_DISCARD
    total = sum(p["m"] for p in reqs)
    with R.rmat_server_create() as s:
        t0 = time.perf_counter()
        report = (lambda done, total: print(f"served {done} of {total} requests", file=sys.stderr, flush=True)) \
            if window_s > 10 else None
        out = R.rmat_server_run_trace(s, reqs, [p["t_arrival"] for p in reqs], report)
        wall = time.perf_counter() - t0
        st = R.rmat_server_get_stats(s)
    assert all(c["status"] == 0 for c in out)
    lat = sorted(c["t_done"] - c["t_submit"] for c in out)
    wait = sorted(c["t_admit"] - c["t_submit"] for c in out)
    pct = lambda v, q: v[min(len(v) - 1, int(q * len(v)))] * 1e3  # noqa: E731
    pooled = f"_pool{pool}" if pool else ""
    res = {"workload": f"served_poisson{rate:g}_k12-28{reading}_ef8-16_var4096{pooled}", "reading": reading,
           "window_s": window_s, "requests": len(reqs), "total_edges": total, "wall_s": wall,
           "edges_per_s": total / wall, "hbm_write_gbs": 8 * total / wall / 1e9,
           "p50_latency_ms": pct(lat, 0.5), "p99_latency_ms": pct(lat, 0.99), "p50_wait_ms": pct(wait, 0.5),
           "p99_wait_ms": pct(wait, 0.99), "table_hit_rate": st["table_hits"] / max(1, st["admitted"]),
           "rounds": st["rounds"], "arena_peak_gb": st["arena_peak"] / 1e9}
    if not plain:
        return res
    # plain per-request launches of the same requests, back to back
    m_max = max(p["m"] for p in reqs)
    src = torch.empty(m_max, dtype=torch.int32, device="cuda")
    dst = torch.empty(m_max, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, p in enumerate(reqs):
        t = R.rmat_build_table_async(p["a"], p["b"], p["c"], p["d"], p["k"], p["table_bound"], p["path_mode"], stream)
        R.rmat_generate_async(t, p["seed"], 0, p["m"], src, dst, stream)
        torch.cuda.synchronize()
        t.close()
        if window_s > 10 and i % 5000 == 4999:
            print(f"plain {i + 1} of {len(reqs)} requests", file=sys.stderr, flush=True)
    plain_s = time.perf_counter() - t0
    del src, dst
    torch.cuda.empty_cache()
    res.update({"plain_edges_per_s": total / plain_s, "served_over_plain": plain_s / wall})
    return res


def k34_chunked(R) -> dict:
    """The k = 34, m = 2^34 instance (a, b, c, d = 0.45, 0.22, 0.22, 0.11,
    variable-length table bounded at 2^16 paths, read from L2; seed 3): all
    16 chunks of 2^30 edges reduced on the device to a 2^16-bin source-prefix
    histogram plus an XOR checksum, timed by HIP events around the 16
    launches; and one 2^28-edge chunk stored as uint64 ids."""
    import torch
    t = R.rmat_build_table(0.45, 0.22, 0.22, 0.11, 34, 1 << 16, R.RMAT_VARIABLE)
    hist = torch.zeros(1 << 16, dtype=torch.int64, device="cuda")
    xr = torch.zeros(1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    R.rmat_generate_reduce_async(t, 3, 0, 1 << 26, 16, hist, xr, stream)  # warm-up
    hist.zero_()
    xr.zero_()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for c in range(16):
        R.rmat_generate_reduce_async(t, 3, c << 30, 1 << 30, 16, hist, xr, stream)
    b.record(stream)
    torch.cuda.synchronize()
    reduce_s = a.elapsed_time(b) / 1e3
    assert int(hist.sum().item()) == 1 << 34
    m = 1 << 28
    src = torch.empty(m, dtype=torch.int64, device="cuda")
    dst = torch.empty(m, dtype=torch.int64, device="cuda")
    R.rmat_generate_async(t, 3, 0, m, src, dst, stream)
    torch.cuda.synchronize()
    a.record(stream)
    R.rmat_generate_async(t, 3, 5 << 30, m, src, dst, stream)
    b.record(stream)
    torch.cuda.synchronize()
    store_s = a.elapsed_time(b) / 1e3
    en, eb = samples_per_edge(R.rmat_table_export(t), 34)
    t.close()
    del src, dst
    torch.cuda.empty_cache()
    from paper_1905_03525_amd.microbench import gather_rate
    ceiling = gather_rate(1 << 20, 16, 2)   # random 16-byte reads from a 1 MB table in L2
    store_rate, reduce_rate = m / store_s, (1 << 34) / reduce_s
    return {"workload": "rmat_k34_m2^34_var65536_l2", "reduce_edges_per_s": reduce_rate,
            "reduce_ms_per_2^30_chunk": reduce_s / 16 * 1e3, "store_edges_per_s": store_rate,
            "store_hbm_write_gbs": 16 * m / store_s / 1e9, "samples_per_edge": en, "philox_blocks_per_edge": eb,
            "roofline": {"bound": "l2_gather", "unit": "reads/s", "peak": ceiling,
                         "peak_source": "measured: random 16-byte reads from a 1 MB device table",
                         "store_achieved": store_rate * en, "store_frac": store_rate * en / ceiling,
                         "reduce_achieved": reduce_rate * en, "reduce_frac": reduce_rate * en / ceiling}}


def k34_degrees(R) -> dict:
    """The k = 34 instance read literally: the out-degree of each of the 2^34
    nodes (2^34 uint32 counters, 64 GiB) over all 2^34 edges, generated in 16
    chunks of 2^30 edges with one atomic increment per edge, then the degree
    distribution (degrees 0 .. 2^20, the last bin clipped), both timed by HIP
    events; checked by its sums (2^34 nodes, 2^34 edges)."""
    import numpy as np
    import torch
    t = R.rmat_build_table(0.45, 0.22, 0.22, 0.11, 34, 1 << 16, R.RMAT_VARIABLE)
    deg = torch.zeros(1 << 34, dtype=torch.int32, device="cuda")
    max_degree = 1 << 20
    hist = torch.zeros(max_degree + 1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    a.record(stream)
    for ch in range(16):
        R.rmat_generate_degrees_async(t, 3, ch << 30, 1 << 30, deg, stream)
    b.record(stream)
    R.rmat_degree_distribution_async(deg, 1 << 34, max_degree, hist, stream)
    c.record(stream)
    torch.cuda.synchronize()
    gen_s, dist_s = a.elapsed_time(b) / 1e3, b.elapsed_time(c) / 1e3
    h = hist.cpu().numpy().view(np.uint64)
    assert int(h.sum()) == 1 << 34 and int(h[-1]) == 0
    assert int((np.arange(max_degree + 1, dtype=np.uint64) * h).sum()) == 1 << 34
    nz = np.nonzero(h)[0]
    t.close()
    del deg, hist
    torch.cuda.empty_cache()
    return {"workload": "rmat_k34_m2^34_var65536_outdegrees", "counters_gib": 64,
            "generate_ms": gen_s * 1e3, "edges_per_s": (1 << 34) / gen_s,
            "distribution_ms": dist_s * 1e3, "distribution_read_gbs": 4 * (1 << 34) / dist_s / 1e9,
            "isolated_nodes": int(h[0]), "max_degree": int(nz[-1]), "degree_1_nodes": int(h[1])}


# ---------------------------------------------------------------------------
# rocprofv3 summaries for profiles/ (each records the command that made it)
#
#   python bench.py summarize trace    OUTDIR              SUMMARY.txt "COMMAND"
#   python bench.py summarize traffic  FETCH_DIR WRITE_DIR SUMMARY.txt "COMMAND"
#   python bench.py summarize counters OUTDIR[,OUTDIR2..]  SUMMARY.txt "COMMAND" [EDGES]
#
# `trace` reads the kernel statistics of `--kernel-trace --stats --output-format
# csv`; `traffic` reads a `--pmc FETCH_SIZE` and a `--pmc WRITE_SIZE` run of
# `bench.py --profile k26` and scales each counter by what it reads for that
# run's 1 GiB copy kernel; `counters` lists any other `--pmc` run per
# dispatch, with per-dispatch rates of the generation kernels.  The traffic
# summary records a hash of the generation kernel's sources; the benchmark
# reports `traffic` only while they match.

KERNEL_SOURCES = ("paper_1905_03525_amd/csrc/generate.hip", "paper_1905_03525_amd/csrc/rmat_internal.h")
GEN_KERNEL = "generate_kernel"
COPY_KERNEL = "copy_kernel"
COPY_BYTES = 1 << 30


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _one(pattern: str, d: str) -> str:
    import glob
    hits = glob.glob(os.path.join(d, "**", pattern), recursive=True)
    if not hits:
        raise FileNotFoundError(f"no {pattern} under {d}")
    return hits[0]


def _counters(d: str) -> dict:
    """{(dispatch, kernel): {counter: value summed over dimensions}}"""
    import csv
    out = {}
    with open(_one("*counter_collection.csv", d)) as f:
        for r in csv.DictReader(f):
            key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
            out.setdefault(key, {})
            out[key][r["Counter_Name"]] = out[key].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return out


def _pick(counters: dict, name_part: str, counter: str) -> float:
    vals = [cs[counter] for (d, k), cs in sorted(counters.items()) if name_part in k and counter in cs]
    if not vals:
        raise KeyError(f"{counter} of {name_part} not found")
    return vals[-1]


def _write(path: str, lines):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize_trace(outdir: str, summary: str, command: str):
    import csv
    rows = list(csv.DictReader(open(_one("*kernel_stats.csv", outdir))))
    lines = ["# rocprofv3 kernel trace statistics", f"# command: {command}", "#",
             "# kernel | calls | total_ns | average_ns | min_ns | max_ns | percent"]
    for r in rows:
        name = r.get("Name", r.get("KERNEL_NAME", "?"))
        lines.append(" | ".join([name[:110], r.get("Calls", "?"), r.get("TotalDurationNs", "?"),
                                 r.get("AverageNs", "?"), r.get("MinNs", "?"), r.get("MaxNs", "?"),
                                 r.get("Percentage", "?")]))
    _write(summary, lines)


def summarize_traffic(fetch_dir: str, write_dir: str, summary: str, command: str):
    fc, wc = _counters(fetch_dir), _counters(write_dir)
    g_fetch, g_write = _pick(fc, GEN_KERNEL, "FETCH_SIZE"), _pick(wc, GEN_KERNEL, "WRITE_SIZE")
    c_fetch, c_write = _pick(fc, COPY_KERNEL, "FETCH_SIZE"), _pick(wc, COPY_KERNEL, "WRITE_SIZE")
    fetch_scale = COPY_BYTES / (c_fetch * 1024.0)
    write_scale = COPY_BYTES / (c_write * 1024.0)
    hbm = g_fetch * 1024.0 * fetch_scale + g_write * 1024.0 * write_scale
    lines = ["# HBM traffic of one generation launch (k=26, 2^30 edges, uint32 ids), rocprofv3 --pmc",
             f"# command: {command}",
             "# counters in KiB per dispatch; scale = known bytes of a 1 GiB copy / what the counter reads for it",
             f"kernel_source_sha256: {kernel_source_hash()}",
             f"generate_fetch_kib: {g_fetch:.1f}", f"generate_write_kib: {g_write:.1f}",
             f"copy_fetch_kib: {c_fetch:.1f}", f"copy_write_kib: {c_write:.1f}",
             f"fetch_scale: {fetch_scale:.4f}", f"write_scale: {write_scale:.4f}",
             f"generate_hbm_bytes: {hbm:.6e}",
             f"algorithmic_bytes: {8 * (1 << 30):.6e}",
             f"traffic_over_algorithmic: {hbm / (8 * (1 << 30)):.4f}"]
    _write(summary, lines)


CU_NUM, N_XCD = 256, 8  # MI355X: 256 compute units in 8 XCDs


def derived_counters(v: dict, edges: float = 0.0) -> dict:
    """rocprofv3's own derived metrics where their counters are present
    (VALUBusy = SQ_ACTIVE_INST_VALU / CU_NUM / GRBM_GUI_ACTIVE, and so on;
    GRBM_GUI_ACTIVE is summed over the XCDs, so one XCD's cycles are the sum
    over N_XCD), and instructions per 64-edge block when the edges of the
    dispatch are given."""
    out = {}
    cyc = v.get("GRBM_GUI_ACTIVE", 0.0) / N_XCD
    if cyc > 0:
        out["gpu_cycles"] = cyc
        for name, num in (("VALUBusy", "SQ_ACTIVE_INST_VALU"), ("SALUBusy", "SQ_INST_CYCLES_SALU"),
                          ("LDSBankConflict", "SQ_LDS_BANK_CONFLICT"), ("LDSActive", "SQ_ACTIVE_INST_LDS"),
                          ("SALUActive", "SQ_ACTIVE_INST_SCA"), ("LDSIdxActive", "SQ_LDS_IDX_ACTIVE"),
                          ("LDSAddrConflict", "SQ_LDS_ADDR_CONFLICT")):
            if num in v:
                out[name] = v[num] / CU_NUM / cyc
    if v.get("SQ_ACTIVE_INST_VALU") and "SQ_THREAD_CYCLES_VALU" in v:
        out["VALUUtilization"] = v["SQ_THREAD_CYCLES_VALU"] / (v["SQ_ACTIVE_INST_VALU"] * 64)
    if "TCC_HIT" in v and "TCC_MISS" in v and v["TCC_HIT"] + v["TCC_MISS"] > 0:
        out["TCC_hit_rate"] = v["TCC_HIT"] / (v["TCC_HIT"] + v["TCC_MISS"])
    if edges > 0:
        blocks = edges / 64
        for n in ("SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_BRANCH", "SQ_INSTS_VMEM_WR",
                  "TCC_REQ", "TCP_TCC_READ_REQ", "TCP_TOTAL_CACHE_ACCESSES"):
            if n in v:
                out[n + "_per_block"] = v[n] / blocks
    return out


def summarize_counters(outdirs: str, summary: str, command: str, edges: str = "0"):
    """outdirs: one or more --pmc output folders (comma-separated) of the same
    program, merged by dispatch; edges: edges of each generation dispatch."""
    merged = {}
    for d in outdirs.split(","):
        for (disp, k), vals in _counters(d).items():
            merged.setdefault((disp, k), {}).update(vals)
    lines = ["# rocprofv3 --pmc counters, summed over XCDs/SEs/CUs, per dispatch; derived as rocprofv3 defines them",
             f"# command: {command}"]
    for (d, k), vals in sorted(merged.items()):
        short = k.split("(")[0][-70:]
        if "generate" in k or "<" in k:
            short = k[:150]
        lines.append(f"{d} {short}: " + ", ".join(f"{n}={v:.6g}" for n, v in sorted(vals.items())))
        der = derived_counters(vals, float(edges) if GEN_KERNEL in k else 0.0)
        if der:
            lines.append(f"{d}   derived: " + ", ".join(f"{n}={v:.4g}" for n, v in sorted(der.items())))
    _write(summary, lines)


def read_traffic(summary: str):
    """Per-launch HBM bytes from a traffic summary, or None if it is missing
    or was taken from different kernel sources."""
    if not os.path.exists(summary):
        return None
    kv = {}
    for ln in open(summary):
        if ":" in ln and not ln.startswith("#"):
            key, v = ln.split(":", 1)
            kv[key.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    return float(kv["generate_hbm_bytes"])


def read_sustained_clock_ghz(summary: str):
    """The mean XCD clock (GHz) that amd-smi sampled while the k = 26
    generation ran back to back (the chip's power limit holds it below the
    rated clock), or None if the summary is missing."""
    if not os.path.exists(summary):
        return None
    for ln in open(summary):
        if ln.startswith("mean_gfx_clock_MHz:"):
            return float(ln.split(":", 1)[1].split()[0]) / 1e3
    return None


def summarize_main(argv) -> int:
    mode = argv[0] if argv else ""
    if mode == "trace" and len(argv) == 4:
        summarize_trace(*argv[1:])
    elif mode == "traffic" and len(argv) == 5:
        summarize_traffic(*argv[1:])
    elif mode == "counters" and len(argv) in (4, 5):
        summarize_counters(*argv[1:])
    else:
        print("usage: bench.py summarize {trace OUT SUMMARY CMD | traffic FETCH WRITE SUMMARY CMD | "
              "counters OUT[,OUT2..] SUMMARY CMD [EDGES]}", file=sys.stderr)
        return 2
    return 0


# ---------------------------------------------------------------------------
# the Sec. 3 generalizations on the k = 26 instance

P3 = [0.3, 0.1, 0.05, 0.1, 0.2, 0.05, 0.05, 0.05, 0.1]  # a 3 x 3 initiator


def _timed(fn, stream, reps: int = 1) -> float:
    """ms of one call of fn() (HIP events on `stream`), after one warm-up
    call; the average of `reps` timed calls."""
    import torch
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def sec3_tables(R, k):
    w = WORKLOAD
    return {
        "epilogue": lambda: R.rmat_build_table(w["a"], w["b"], w["c"], w["d"], k, w["table_bound"], R.RMAT_VARIABLE),
        # degree smoothing: 8 perturbed tables of bound 1024 (eps 0.1), edge e
        # from table e mod 8; the whole set stays LDS-resident
        "perturbed": lambda: R.rmat_build_perturbed_table(w["a"], w["b"], w["c"], w["d"], k, 1024, R.RMAT_VARIABLE,
                                                          8, 0.1, 2019),
        # 3^17 = 1.29e8 nodes (uint32 ids), a 4096-bound table
        "kron3x3": lambda: R.rmat_kron_build_table(P3, 3, 17, 4096, R.RMAT_VARIABLE),
    }


def sec3_launch(R, which, t, src, dst, stream):
    w = WORKLOAD
    if which == "epilogue":  # undirected mirror + id scramble
        return lambda: R.rmat_generate_ex_async(t, w["seed"], 0, w["m"], 3, 0x5EED, src, dst, stream)
    return lambda: R.rmat_generate_async(t, w["seed"], 0, w["m"], src, dst, stream)


def sec3_measurements(R, src, dst, stream, ops_per_edge: float) -> dict:
    """The epilogue, the perturbed set, the 3 x 3 Kronecker initiator and
    partitioned generation on the k = 26 instance's 2^30 edges."""
    w = WORKLOAD
    k, m = w["k"], w["m"]
    out = {}
    tabs = sec3_tables(R, k)
    t = tabs["epilogue"]()
    ms = _timed(sec3_launch(R, "epilogue", t, src, dst, stream), stream)
    t.close()
    out["undirected_scrambled_kernel_ms"] = ms
    out["undirected_scrambled_roofline"] = alu_roofline(ms, m, ops_per_edge + OPS_EPILOGUE)
    out["undirected_scrambled_edges_per_s"] = m / (ms / 1e3)
    t = tabs["perturbed"]()
    ms = _timed(sec3_launch(R, "perturbed", t, src, dst, stream), stream)
    laws = [samples_per_edge(R.rmat_table_export_member(t, i), k) for i in range(8)]
    t.close()
    en_set = sum(x[0] for x in laws) / 8  # edge e uses member e mod 8
    eb_set = sum(x[1] for x in laws) / 8
    out["perturbed_set"] = {"tables": 8, "table_bound": 1024, "epsilon": 0.1, "kernel_ms": ms,
                            "edges_per_s": m / (ms / 1e3), "samples_per_edge": en_set,
                            "philox_blocks_per_edge": eb_set,
                            "roofline": alu_roofline(ms, m, eb_set * OPS_PER_PHILOX_BLOCK + en_set * OPS_PER_SAMPLE)}
    t = tabs["kron3x3"]()
    ms = _timed(sec3_launch(R, "kron3x3", t, src, dst, stream), stream)
    en_k, eb_k = samples_per_edge(R.rmat_table_export(t), 17)  # letters are digit pairs
    t.close()
    b0 = time.perf_counter()
    tk = tabs["kron3x3"]()
    kron_build_ms = (time.perf_counter() - b0) * 1e3
    tk.close()
    out["kronecker_3x3"] = {"k": 17, "nodes": 3 ** 17, "table_bound": 4096, "kernel_ms": ms,
                            "edges_per_s": m / (ms / 1e3), "samples_per_edge": en_k, "philox_blocks_per_edge": eb_k,
                            "table_build_ms": kron_build_ms,
                            "roofline": alu_roofline(ms, m, eb_k * OPS_PER_PHILOX_BLOCK + en_k * OPS_PER_SAMPLE +
                                                     OPS_KRON_CUT)}
    # partitioned generation of the same instance: 2^8 x 2^8 tiles, tile
    # rows [0, 64) per call, four calls enqueued on one stream; each range is
    # counted on the host while the previous one generates (counting included)
    t_part = R.rmat_build_table(w["a"], w["b"], w["c"], w["d"], k, w["table_bound"], R.RMAT_VARIABLE)
    import torch
    stream = torch.cuda.current_stream()

    def partitioned(times=None):
        n_all = 0
        for r0 in range(0, 256, 64):
            c0 = time.perf_counter()
            n = int(R.rmat_partition_counts(t_part, w["seed"], m, 8, r0, r0 + 64).sum())
            if times is not None:
                times.append(time.perf_counter() - c0)
            R.rmat_generate_partition_async(t_part, w["seed"], m, 8, r0, r0 + 64, src[n_all:], dst[n_all:], n,
                                            stream)
            n_all += n
        torch.cuda.synchronize()
        return n_all

    partitioned()  # warm-up (list buffers, code objects)
    count_times = []
    p0 = time.perf_counter()
    n_part = partitioned(count_times)
    part_s = time.perf_counter() - p0
    assert n_part == m
    out["partitioned_edges_per_s"] = m / part_s
    out["partitioned_config"] = {"tile_bits": 8, "row_ranges": 4, "total_ms": part_s * 1e3,
                                 "host_count_ms": sum(count_times) * 1e3,
                                 "first_count_ms": count_times[0] * 1e3, "overlapped": True}
    t_part.close()
    return out


# ---------------------------------------------------------------------------
# profiling targets: one workload's launches and nothing else, then a 1 GiB
# device copy of known traffic (read 1 GiB, write 1 GiB) to scale the HBM
# byte counters of the same run

PROFILE_TARGETS = ("k26", "epilogue", "perturbed", "kron3x3", "k34_store", "k34_reduce", "microbench")


def profile_main(R, what: str, steps: int, warmup: int) -> dict:
    import torch
    from paper_1905_03525_amd import microbench
    from paper_1905_03525_amd.rmat import _check
    w = WORKLOAD
    stream = torch.cuda.current_stream()
    ran = {"profile": what, "steps": steps, "warmup": warmup}
    if what in ("k26", "epilogue", "perturbed", "kron3x3"):
        m = w["m"]
        src = torch.empty(m, dtype=torch.int32, device="cuda")
        dst = torch.empty(m, dtype=torch.int32, device="cuda")
        if what == "k26":
            t = R.rmat_build_table(w["a"], w["b"], w["c"], w["d"], w["k"], w["table_bound"], R.RMAT_VARIABLE)
            fn = lambda: R.rmat_generate_async(t, w["seed"], 0, m, src, dst, stream)  # noqa: E731
        else:
            t = sec3_tables(R, w["k"])[what]()
            fn = sec3_launch(R, what, t, src, dst, stream)
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ran["kernel_ms"] = _timed(fn, stream, max(1, steps)) if steps else None
        t.close()
        del src, dst
    elif what in ("k34_store", "k34_reduce"):
        t = R.rmat_build_table(0.45, 0.22, 0.22, 0.11, 34, 1 << 16, R.RMAT_VARIABLE)
        m = 1 << 28
        if what == "k34_store":
            src = torch.empty(m, dtype=torch.int64, device="cuda")
            dst = torch.empty(m, dtype=torch.int64, device="cuda")
            fn = lambda: R.rmat_generate_async(t, 3, 5 << 30, m, src, dst, stream)  # noqa: E731
        else:
            hist = torch.zeros(1 << 16, dtype=torch.int64, device="cuda")
            xr = torch.zeros(1, dtype=torch.int64, device="cuda")
            fn = lambda: R.rmat_generate_reduce_async(t, 3, 5 << 30, m, 16, hist, xr, stream)  # noqa: E731
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ran["kernel_ms"] = _timed(fn, stream, max(1, steps)) if steps else None
        ran["edges"] = m
        t.close()
    elif what == "microbench":
        # the ceilings: random 16/8/4-byte LDS reads, random 16-byte L2 gathers
        out = torch.zeros(1, dtype=torch.int64, device="cuda")
        for width in (16, 8, 4):
            _check(microbench._lib().rmat_bench_lds_read(1 << 12, 65536, width, out.data_ptr(), None),
                     "rmat_bench_lds_read")
        ran["gather_reads_per_s"] = microbench.gather_rate(1 << 20, 16, 2)
        torch.cuda.synchronize()
    else:
        raise SystemExit(f"--profile takes one of {PROFILE_TARGETS}")
    torch.cuda.empty_cache()
    a = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    b = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    _check(microbench._lib().rmat_bench_copy(a.data_ptr(), b.data_ptr(), COPY_BYTES, None), "rmat_bench_copy")
    torch.cuda.synchronize()
    ran["copy_bytes"] = COPY_BYTES
    return ran


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "summarize":
        sys.exit(summarize_main(sys.argv[2:]))
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-instance batched comparison")
    ap.add_argument("--served-window", type=float, default=60.0,
                    help="seconds of the 2000 requests/s stream to serve (0: skip; the full stream is 60)")
    ap.add_argument("--served-plain-window", type=float, default=3.0,
                    help="seconds of the stream served again and then generated by plain launches (0: skip)")
    ap.add_argument("--served-reading", default="A", choices=["A", "B"])
    ap.add_argument("--served-no-plain", action="store_true", help="skip the plain-launch comparison of the stream")
    ap.add_argument("--served-pool", type=int, default=0,
                    help="also run the stream window with parameters from this many pre-drawn sets (cache hits)")
    ap.add_argument("--no-k34", action="store_true", help="skip the k=34 chunked instance")
    ap.add_argument("--no-sec3", action="store_true",
                    help="skip the epilogue, perturbed-set, Kronecker and partitioned measurements")
    ap.add_argument("--profile", choices=PROFILE_TARGETS,
                    help="profiling target: only this workload's launches (--warmup untimed, --steps timed), then "
                         "a 1 GiB copy that calibrates the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the sampler needs no second one "
                                   "(edges of disjoint index ranges are generated independently)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1905_03525_amd as R

    torch.cuda.set_device(0)
    if args.profile:
        print(json.dumps(profile_main(R, args.profile, args.steps, args.warmup)), flush=True)
        return
    w = WORKLOAD
    k, m = w["k"], w["m"]
    stream = torch.cuda.current_stream()
    src = torch.empty(m, dtype=torch.int32, device="cuda")
    dst = torch.empty(m, dtype=torch.int32, device="cuda")

    def step(events=None):
        # the table is built on the device on the same stream, then the edges
        # generated from it: the host waits for neither
        t = R.rmat_build_table_async(w["a"], w["b"], w["c"], w["d"], k, w["table_bound"], R.RMAT_VARIABLE, stream)
        if events is not None:
            events[0].record(stream)
        R.rmat_generate_async(t, w["seed"], 0, m, src, dst, stream)
        if events is not None:
            events[1].record(stream)
        return t

    tables = []
    for _ in range(args.warmup):
        tables.append(step())
    torch.cuda.synchronize()
    for t in tables:
        t.close()
    tables = []

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        tables.append(step(ev[i]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for t in tables:
        t.close()

    kern_ms = [a.elapsed_time(b) for a, b in ev]
    avg_kern_s = sum(kern_ms) / len(kern_ms) / 1e3
    build_t0 = time.perf_counter()
    tb = R.rmat_build_table(w["a"], w["b"], w["c"], w["d"], k, w["table_bound"], R.RMAT_VARIABLE)
    build_ms = (time.perf_counter() - build_t0) * 1e3
    info = R.rmat_table_info(tb)
    en, eb = samples_per_edge(R.rmat_table_export(tb), k)
    tb.close()

    traffic = read_traffic(TRAFFIC_SUMMARY)
    clock_ghz = read_sustained_clock_ghz(POWER_CLOCK_SUMMARY)
    value = m * args.steps / wall
    ops_per_edge = eb * OPS_PER_PHILOX_BLOCK + en * OPS_PER_SAMPLE
    achieved_ops = ops_per_edge * m / avg_kern_s
    hbm_gbs = BYTES_PER_EDGE * m / avg_kern_s / 1e9
    out = {
        "metric": "edges/s & HBM write GB/s (k=26, ef16); batched vs per-instance speedup",
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w["name"], "k": k, "m": m, "edge_factor": 16, "a": w["a"], "b": w["b"], "c": w["c"],
                   "d": w["d"], "table_bound": w["table_bound"], "path_mode": w["path_mode"], "seed": w["seed"],
                   "id_bits": 32, "n_items": info["n_items"], "expected_len": info["expected_len"]},
        "hbm_write_gbs": BYTES_PER_EDGE * value / 1e9,
        "generate_kernel_ms": avg_kern_s * 1e3,
        "generate_kernel_hbm_write_gbs": hbm_gbs,
        "generate_kernel_hbm_frac": hbm_gbs / HBM_PEAK_GBS,
        "write_stream_gbs": None,
        "generate_kernel_write_stream_frac": None,
        "table_build_ms": build_ms,
        "samples_per_edge": en,
        "philox_blocks_per_edge": eb,
        "roofline": {"bound": "alu", "achieved": achieved_ops / 1e12, "peak": INT_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved_ops / INT_PEAK_OPS,
                     "ops_per_edge": ops_per_edge,
                     "traffic": traffic,
                     # the same peak at the clock the power limit leaves on this kernel
                     "sustained_clock_ghz": clock_ghz,
                     "frac_at_sustained_clock": (achieved_ops / (INT_PEAK_OPS * clock_ghz / PEAK_CLOCK_GHZ)
                                                 if clock_ghz else None)},
    }
    print(f"k=26 steps done: {out['generate_kernel_ms']:.3f} ms per generation", file=sys.stderr, flush=True)
    # the measured store-only stream on this device: the achievable write
    # ceiling the id stores are compared with beside the 8 TB/s spec
    from paper_1905_03525_amd import microbench
    del src, dst
    torch.cuda.empty_cache()
    ws = microbench.write_bandwidth()
    out["write_stream_gbs"] = ws
    out["generate_kernel_write_stream_frac"] = hbm_gbs / ws
    if not args.no_sec3:
        src = torch.empty(m, dtype=torch.int32, device="cuda")
        dst = torch.empty(m, dtype=torch.int32, device="cuda")
        out.update(sec3_measurements(R, src, dst, stream, ops_per_edge))
        del src, dst
        torch.cuda.empty_cache()
        print("Sec. 3 measurements done", file=sys.stderr, flush=True)
    if not args.no_batch:
        bt = batched_vs_plain(R)
        out["batched_speedup"] = bt["speedup"]
        out["batched"] = bt
        print("batched workload done", file=sys.stderr, flush=True)
    if not args.no_k34:
        out["k34"] = k34_chunked(R)
        out["k34_degrees"] = k34_degrees(R)
        print("k=34 workloads done", file=sys.stderr, flush=True)
    if args.served_window > 0:
        # the whole stream through the server; the comparison with plain
        # per-request launches on a shorter window of it (the plain
        # launches of the full minute would take several more minutes)
        out["served"] = served_vs_plain(R, args.served_window, args.served_reading, plain=False)
    if args.served_plain_window > 0 and not args.served_no_plain:
        out["served_vs_plain"] = served_vs_plain(R, args.served_plain_window, args.served_reading, plain=True)
    if args.served_pool > 0:
        out["served_pooled"] = served_vs_plain(R, args.served_plain_window or 3.0, args.served_reading,
                                               plain=not args.served_no_plain, pool=args.served_pool)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
