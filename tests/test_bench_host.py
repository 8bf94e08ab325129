"""Host-side pieces of the benchmark: the exact samples-per-edge law it
prices the roofline with, and its refusal of more than one GPU."""
from __future__ import annotations

import importlib.util
import os
import subprocess
import sys

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_samples_per_edge_matches_simulation():
    """E[N] and E[ceil(N/4)] from the renewal law equal the counts the oracle
    reports edge by edge (k = 26, the benchmark's 4096-entry table)."""
    b = _bench()
    t = oracle.build_table(0.57, 0.19, 0.19, 0.05, 26, 4096, oracle.VARIABLE)
    exp = {"len": t.length.astype(np.uint32), "w": t.w.astype(np.uint64)}
    en, eb = b.samples_per_edge(exp, 26)
    _, _, ns = oracle.generate(t, 7, 0, 1 << 18, threads=8, samples=True)
    assert abs(ns.mean() - en) < 4 * ns.std() / np.sqrt(ns.size)
    blocks = (ns.astype(np.int64) + 3) // 4
    assert abs(blocks.mean() - eb) < 4 * blocks.std() / np.sqrt(blocks.size)
    assert abs(en - 4.0200) < 1e-3 and abs(eb - 1.1091) < 1e-3


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode != 0
    assert '"n_gpus": 2' in r.stdout and "one GPU" in r.stdout
