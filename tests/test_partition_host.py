"""The library's host-side tile counting (partitioned generation, Sec. 3)
compiled with g++ against the fake device of tests/hostsim and compared,
count for count, with the oracle: both take every integer decision of the
binomial draws from the same sequence of floating-point operations."""
from __future__ import annotations

import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIM = os.path.join(ROOT, "tests", "hostsim")
CSRC = os.path.join(ROOT, "paper_1905_03525_amd", "csrc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("partsim") / "libpartsim.so")
    cmd = ["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
           "-I", SIM, "-I", os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(CSRC, "api.cpp"),
           os.path.join(CSRC, "partition.cpp"), os.path.join(SIM, "fake_device.cpp"), "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    L = ctypes.CDLL(out)
    vp, u64 = ctypes.c_void_p, ctypes.c_uint64
    L.rmat_build_table.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, u64, ctypes.c_int, ctypes.POINTER(vp)]
    L.rmat_partition_counts.argtypes = [vp, u64, u64, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, vp]
    L.rmat_free_table.argtypes = [vp]
    L.rmat_generate_partition.argtypes = [vp, u64, u64, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, vp, vp, u64]
    L.rmat_generate_partition_async.argtypes = [vp, u64, u64, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, vp, vp,
                                                u64, vp]
    L.sim_whole_cover.argtypes = [ctypes.c_int]
    L.sim_cover_insts.restype = u64
    L.rmat_last_error.restype = ctypes.c_char_p
    return L


CASES = [
    # q, k, bound, seed, m, tile_bits, rows
    ((0.57, 0.19, 0.19, 0.05), 12, 256, 3, 100_000, 3, None),
    ((0.57, 0.19, 0.19, 0.05), 26, 4096, 7, 1 << 30, 6, None),
    ((0.45, 0.22, 0.22, 0.11), 34, 1 << 16, 3, 1 << 34, 8, (17, 90)),
    ((0.25, 0.25, 0.25, 0.25), 40, 1000, 11, 2 ** 53, 9, (500, 512)),
    ((0.9, 0.025, 0.025, 0.05), 30, 8192, 12, 10 ** 12, 7, (0, 3)),
    ((1.0, 0.0, 0.0, 0.0), 20, 300, 1, 123_456, 4, None),
    ((0.5, 0.5, 0.0, 0.0), 20, 300, 2, 7, 5, None),
    ((0.6, 0.1, 0.3, 0.0), 16, 64, 5, 0, 2, None),
    ((0.57, 0.19, 0.19, 0.05), 64, 4096, 2 ** 64 - 1, 10 ** 15, 15, (32767, 32768)),
]


@pytest.mark.parametrize("q,k,bound,seed,m,tb,rows", CASES)
def test_library_counts_equal_oracle(lib, q, k, bound, seed, m, tb, rows):
    r0, r1 = rows if rows else (0, 1 << tb)
    h = ctypes.c_void_p()
    assert lib.rmat_build_table(*q, k, bound, 1, ctypes.byref(h)) == 0, lib.rmat_last_error()
    got = np.zeros((r1 - r0, 1 << tb), np.uint64)
    assert lib.rmat_partition_counts(h, seed, m, tb, r0, r1, got.ctypes.data_as(ctypes.c_void_p)) == 0, \
        lib.rmat_last_error()
    lib.rmat_free_table(h)
    t = oracle.build_table(*q, k, bound, oracle.VARIABLE)
    want = oracle.partition_counts(t, seed, m, tb, r0, r1)
    assert np.array_equal(got, want)
    if rows is None:
        assert int(got.sum()) == m


LIST_CASES = [
    # q, k, bound, seed, m, tile_bits, rows: big tiles cut into several items,
    # small ones packed (pack limits by instance count and by blocks), 64-bit ids
    ((0.57, 0.19, 0.19, 0.05), 26, 4096, 7, 1 << 30, 6, None),
    ((0.57, 0.19, 0.19, 0.05), 24, 4096, 5, 1 << 22, 10, (0, 4)),
    ((0.25, 0.25, 0.25, 0.25), 20, 1000, 3, 1 << 22, 8, (0, 16)),   # tiles of 64 edges: 256 per pack
    ((0.25, 0.25, 0.25, 0.25), 22, 1000, 4, 450 << 16, 8, (7, 9)),  # tiles of 7-8 blocks: packs end by blocks
    ((0.45, 0.22, 0.22, 0.11), 34, 1 << 16, 3, 1 << 30, 8, (17, 20)),
]


@pytest.mark.parametrize("q,k,bound,seed,m,tb,rows", LIST_CASES)
def test_generation_lists_cover_every_tile_once(lib, q, k, bound, seed, m, tb, rows):
    """The tile list of a partitioned generation (through the fake device):
    one instance per non-empty tile, all on one table, with running block
    counts; the waves' parts, cut and searched as the kernel does for several
    grid sizes, hold every block of every tile exactly once."""
    r0, r1 = rows if rows else (0, 1 << tb)
    h = ctypes.c_void_p()
    assert lib.rmat_build_table(*q, k, bound, 1, ctypes.byref(h)) == 0, lib.rmat_last_error()
    counts = np.zeros((r1 - r0, 1 << tb), np.uint64)
    assert lib.rmat_partition_counts(h, seed, m, tb, r0, r1, counts.ctypes.data_as(ctypes.c_void_p)) == 0
    out = np.zeros(2, np.uint64)   # the fake device writes no ids
    p = out.ctypes.data_as(ctypes.c_void_p)
    lib.sim_whole_cover(1)
    try:
        rc = lib.rmat_generate_partition(h, seed, m, tb, r0, r1, p, p, int(counts.sum()))
        assert rc == 0, lib.rmat_last_error()
        assert lib.sim_failed() == 0
        assert lib.sim_cover_insts() == int((counts > 0).sum())
    finally:
        lib.sim_whole_cover(0)
        lib.rmat_free_table(h)


def test_async_calls_wrap_the_list_ring(lib):
    """Asynchronous partitioned generations through the fake device: seven
    calls in a row (the ring holds four list buffers, so the later ones wait
    for earlier launches and reuse their buffers, grown when a range has more
    tiles), every tile list covered exactly once."""
    q, k, tb, m, seed = (0.57, 0.19, 0.19, 0.05), 20, 6, 1 << 20, 4
    h = ctypes.c_void_p()
    assert lib.rmat_build_table(*q, k, 4096, 1, ctypes.byref(h)) == 0, lib.rmat_last_error()
    out = np.zeros(2, np.uint64)
    p = out.ctypes.data_as(ctypes.c_void_p)
    lib.sim_whole_cover(1)
    try:
        for r0, r1 in [(0, 2), (2, 3), (3, 30), (30, 31), (31, 33), (33, 64), (0, 64)]:
            counts = np.zeros((r1 - r0, 1 << tb), np.uint64)
            assert lib.rmat_partition_counts(h, seed, m, tb, r0, r1, counts.ctypes.data_as(ctypes.c_void_p)) == 0
            rc = lib.rmat_generate_partition_async(h, seed, m, tb, r0, r1, p, p, int(counts.sum()), None)
            assert rc == 0, lib.rmat_last_error()
            assert lib.sim_failed() == 0
            assert lib.sim_cover_insts() == int((counts > 0).sum())
    finally:
        lib.sim_whole_cover(0)
        lib.rmat_free_table(h)


def test_list_ring_settles_for_calls_of_varying_sizes(lib):
    """Calls of varying sizes rotating through the ring of four list buffers
    (five row ranges per pass, so each pass puts them on other buffers): a
    buffer that grows takes at least twice its size and the ring's largest,
    so each buffer grows at most twice (its first size, then the largest
    range's) and the ring stops allocating once every buffer has met it."""
    # more non-empty tiles than any other test here lists, so that the ring
    # grows whatever ran before in this process
    q, k, tb, m, seed = (0.57, 0.19, 0.19, 0.05), 20, 8, 1 << 24, 5
    lib.sim_mallocs.restype = ctypes.c_uint64
    h = ctypes.c_void_p()
    assert lib.rmat_build_table(*q, k, 4096, 1, ctypes.byref(h)) == 0, lib.rmat_last_error()
    out = np.zeros(2, np.uint64)
    p = out.ctypes.data_as(ctypes.c_void_p)
    ranges = [(0, 4), (4, 128), (128, 130), (130, 256), (0, 256)]
    try:
        per_pass = []
        for _ in range(6):
            before = lib.sim_mallocs()
            for r0, r1 in ranges:
                counts = np.zeros((r1 - r0, 1 << tb), np.uint64)
                assert lib.rmat_partition_counts(h, seed, m, tb, r0, r1, counts.ctypes.data_as(ctypes.c_void_p)) == 0
                rc = lib.rmat_generate_partition_async(h, seed, m, tb, r0, r1, p, p, int(counts.sum()), None)
                assert rc == 0, lib.rmat_last_error()
                assert lib.sim_failed() == 0
            per_pass.append(lib.sim_mallocs() - before)
        # a growth allocates the device buffer and its pinned twin
        assert per_pass[0] > 0 and per_pass[-2:] == [0, 0], per_pass
        assert sum(per_pass) <= 2 * 2 * 4, per_pass
    finally:
        lib.rmat_free_table(h)
