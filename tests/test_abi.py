"""CPU checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid tables before touching a device."""
from __future__ import annotations

import os
import re

import pytest

import paper_1905_03525_amd as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(rmat\w*)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    L = R.load()
    declared = _declared()
    assert declared, "no declarations found"
    missing = [n for n in sorted(declared) if not hasattr(L, n)]
    assert not missing, missing
    assert set(R.rmat.EXPORTED) <= declared


@pytest.mark.parametrize("args", [
    (0.5, 0.5, 0.1, -0.1, 10, 100, R.RMAT_VARIABLE),
    (0.5, 0.2, 0.2, 0.2, 10, 100, R.RMAT_VARIABLE),
    (0.25, 0.25, 0.25, 0.25, 0, 100, R.RMAT_VARIABLE),
    (0.25, 0.25, 0.25, 0.25, 65, 100, R.RMAT_VARIABLE),
    (0.25, 0.25, 0.25, 0.25, 10, 4, R.RMAT_VARIABLE),
    (0.25, 0.25, 0.25, 0.25, 10, 3, R.RMAT_FIXED),
    (0.25, 0.25, 0.25, 0.25, 2, 256, R.RMAT_FIXED),
    (0.25, 0.25, 0.25, 0.25, 20, 2**24 + 1, R.RMAT_VARIABLE),
    (0.25, 0.25, 0.25, 0.25, 20, 100, 2),
    (float("nan"), 0.5, 0.25, 0.25, 10, 100, R.RMAT_VARIABLE),
    (float("inf"), 0.5, 0.25, 0.25, 10, 100, R.RMAT_VARIABLE),
])
def test_invalid_tables_rejected_on_host(args):
    with pytest.raises(R.RmatError) as ei:
        R.rmat_build_table(*args)
    assert ei.value.status == R.RMAT_EINVAL
    assert R.rmat_last_error()


def test_null_handles():
    import ctypes
    L = R.load()
    assert L.rmat_free_table(None) == R.RMAT_OK
    assert L.rmat_generate(None, 1, 0, 10, None, None) == R.RMAT_EINVAL
    assert L.rmat_table_info(None, None) == R.RMAT_EINVAL
    assert L.rmat_table_export(None, None, 0) == R.RMAT_EINVAL
    assert L.rmat_build_table(0.25, 0.25, 0.25, 0.25, 10, 100, 1, ctypes.cast(0, ctypes.POINTER(ctypes.c_void_p))) \
        == R.RMAT_EINVAL


def _inst(**kw):
    p = dict(a=0.57, b=0.19, c=0.19, d=0.05, k=16, path_mode=R.RMAT_VARIABLE, table_bound=256, seed=1,
             edge_begin=0, m=0, out_src=None, out_dst=None)
    p.update(kw)
    return p


@pytest.mark.parametrize("bad,status", [
    (dict(k=0), R.RMAT_EINVAL),
    (dict(a=0.6), R.RMAT_EINVAL),
    (dict(table_bound=3), R.RMAT_EINVAL),
    (dict(path_mode=R.RMAT_FIXED, table_bound=4 ** 6, k=4), R.RMAT_EINVAL),
    (dict(m=10), R.RMAT_EINVAL),                                  # NULL outputs
    (dict(m=10, out_src=6, out_dst=8), R.RMAT_EINVAL),            # 6 not 4-byte aligned
    (dict(m=10, k=40, out_src=12, out_dst=16), R.RMAT_EINVAL),    # 64-bit ids need 8-byte alignment
    (dict(m=2, edge_begin=2 ** 64 - 1, out_src=16, out_dst=32), R.RMAT_ERANGE),
])
def test_batch_invalid_instance_rejected_on_host(bad, status):
    insts = [_inst(), _inst(seed=2), _inst(**bad)]
    with pytest.raises(R.RmatError) as ei:
        R.rmat_batch_create(insts)
    assert ei.value.status == status
    assert "instance 2" in str(ei.value)


def test_batch_null_handles():
    import ctypes
    L = R.load()
    assert L.rmat_batch_free(None) == R.RMAT_OK
    assert L.rmat_batch_enqueue(None, None) == R.RMAT_EINVAL
    assert L.rmat_batch_launch_graph(None, None) == R.RMAT_EINVAL
    assert L.rmat_batch_check(None) == R.RMAT_EINVAL
    assert L.rmat_batch_get_info(None, None) == R.RMAT_EINVAL
    assert L.rmat_batch_table_info(None, 0, None) == R.RMAT_EINVAL
    assert L.rmat_batch_table_export(None, 0, None, 0) == R.RMAT_EINVAL
    assert L.rmat_batch_create(None, 0, 0, ctypes.cast(0, ctypes.POINTER(ctypes.c_void_p))) == R.RMAT_EINVAL
    assert L.rmat_batch_autotune(None, 0, None) == R.RMAT_EINVAL


def test_autotune_rejects_invalid_instance_on_host():
    with pytest.raises(R.RmatError) as ei:
        R.rmat_batch_autotune([_inst(table_bound=0), _inst(table_bound=0, b=0.5)])
    assert ei.value.status == R.RMAT_EINVAL and "instance 1" in str(ei.value)


def test_server_null_handles_and_config_checks():
    import ctypes
    L = R.load()
    assert L.rmat_server_free(None) == R.RMAT_OK
    assert L.rmat_server_submit(None, None, -1.0, None) == R.RMAT_EINVAL
    assert L.rmat_server_step(None, None) == R.RMAT_EINVAL
    assert L.rmat_server_drain(None) == R.RMAT_EINVAL
    assert L.rmat_server_poll(None, None, 0, None) == R.RMAT_EINVAL
    assert L.rmat_server_release(None, 1) == R.RMAT_EINVAL
    assert L.rmat_server_run_trace(None, None, None, 0, None, R.rmat.PROGRESS_FN(), None) == R.RMAT_EINVAL
    assert L.rmat_server_get_stats(None, None) == R.RMAT_EINVAL
    assert L.rmat_server_clock(None) == 0.0
    assert L.rmat_server_create(None, ctypes.cast(0, ctypes.POINTER(ctypes.c_void_p))) == R.RMAT_EINVAL
    for bad in (dict(table_slots=4, max_active=8), dict(max_table_bound=3), dict(max_inflight=9)):
        with pytest.raises(R.RmatError) as ei:
            R.rmat_server_create(**bad)
        assert ei.value.status == R.RMAT_EINVAL


def test_perturbed_set_member_size_rejected_on_host():
    """A perturbed set of more than one table takes member tables of at most
    2^19 buckets (a member's byte offset is a 24-bit product); the check
    runs on the host, before any device call."""
    with pytest.raises(R.RmatError) as ei:
        R.rmat_build_perturbed_table(0.57, 0.19, 0.19, 0.05, 30, 1 << 20, R.RMAT_VARIABLE, 2, 0.1, 7)
    assert ei.value.status == R.RMAT_EINVAL
    assert "2^19" in R.rmat_last_error()
