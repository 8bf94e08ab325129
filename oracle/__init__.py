"""CPU oracle for the linear-work R-MAT sampler (arXiv 1905.03525).

TEST INFRASTRUCTURE ONLY.  The product library never imports, links or calls
this package; only the test suite, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP implementation.

The arithmetic lives in ``rmat_oracle.c`` (plain C, compiled with gcc); this
module compiles it on demand and exposes it through ctypes with numpy arrays.
The header comment of ``rmat_oracle.c`` lists the passages of the paper each
step follows and the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rmat_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FIXED = 0
VARIABLE = 1

_ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EINTERNAL", -4: "ERANGE"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed: {_ERRORS.get(code, code)}")
        self.code = code
        self.name = _ERRORS.get(code, str(code))


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (no fused multiply-add: the canonical
    products must round after every multiplication)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-pthread", "-Wall", "-Wno-unused-function",
            _SRC, "-o", tmp, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x32_10.restype = None
        L.orc_canonical_product.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        L.orc_canonical_product.restype = ctypes.c_double
        L.orc_table_new.restype = ctypes.c_void_p
        L.orc_table_delete.argtypes = [ctypes.c_void_p]
        L.orc_build_table.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
        L.orc_build_table.restype = ctypes.c_int
        L.orc_table_info.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.orc_table_arrays.argtypes = [ctypes.c_void_p] + [ctypes.c_void_p] * 8
        L.orc_generate.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
        L.orc_generate.restype = ctypes.c_int
        L.orc_generate_reduce.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        L.orc_generate_reduce.restype = ctypes.c_int
        L.orc_edge_mix.argtypes = [ctypes.c_uint64] * 3
        L.orc_edge_mix.restype = ctypes.c_uint64
        L.orc_generate_ex.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_uint64]
        L.orc_generate_ex.restype = ctypes.c_int
        L.orc_scramble.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64]
        L.orc_scramble.restype = ctypes.c_uint64
        L.orc_kron_build_table.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int,
                                           ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p]
        L.orc_kron_build_table.restype = ctypes.c_int
        L.orc_perturbed_params.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                                                   ctypes.c_void_p]
        L.orc_perturbed_params.restype = ctypes.c_int
        L.orc_generate_set.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
                                       ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        L.orc_generate_set.restype = ctypes.c_int
        L.orc_binomial.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_uint64,
                                   ctypes.c_double]
        L.orc_binomial.restype = ctypes.c_uint64
        L.orc_partition_counts.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                           ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]
        L.orc_partition_counts.restype = ctypes.c_int
        L.orc_generate_partition.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int,
                                             ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int, ctypes.c_void_p]
        L.orc_generate_partition.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 (Salmon et al., SC'11): 4 output words for one counter."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def canonical_product(q, counts) -> float:
    """Probability of a path with the given letter counts (reading R3)."""
    qa = (ctypes.c_double * 4)(*[float(v) for v in q])
    ca = (ctypes.c_int * 4)(*[int(v) for v in counts])
    return float(lib().orc_canonical_product(qa, ca))


def scramble(k: int, key: int, x: int) -> int:
    """The scramble bijection pi of [0, 2^k) under `key` (reading R19)."""
    return int(lib().orc_scramble(k, key, x))


def edge_mix(e: int, src: int, dst: int) -> int:
    return int(lib().orc_edge_mix(e, src, dst))


@dataclass
class Table:
    """An oracle table: items in tree order, then the alias buckets."""
    k: int
    mode: int
    cap: int
    bucket_bits: int
    n_items: int
    n_buckets: int
    capacity: int
    length: np.ndarray   # uint8, per item (padding items: 0)
    code: np.ndarray     # uint64, base-4 path code, root-most letter first
    row: np.ndarray      # uint32, row bits of the path (root-most = MSB)
    col: np.ndarray      # uint32
    p: np.ndarray        # float64, canonical product
    w: np.ndarray        # int64, fixed-point weight (sum = 2^32)
    thr: np.ndarray      # uint32, per bucket
    alias: np.ndarray    # uint32, per bucket
    handle: "ctypes.c_void_p" = None
    K: int = 2           # initiator size (2: R-MAT; K > 2: base-K digits, K^2-ary codes)

    def __del__(self):
        if self.handle is not None and _lib is not None:
            _lib.orc_table_delete(self.handle)
            self.handle = None

    @property
    def expected_len(self) -> float:
        """Mean path length under the quantised law, sum(w L) / 2^32."""
        return float(np.sum(self.w.astype(np.float64) * self.length) / 2.0**32)


def build_table(a, b, c, d, k, bound, mode) -> Table:
    L = lib()
    h = L.orc_table_new()
    rc = L.orc_build_table(a, b, c, d, int(k), int(bound), int(mode), h)
    if rc != 0:
        L.orc_table_delete(h)
        raise OracleError(rc, "build_table")
    return _wrap_table(h)


def kron_build_table(P, K: int, k: int, bound: int, mode: int) -> Table:
    """Table of a K x K initiator P (K^2 probabilities, row-major; cell
    (i, j) is letter K i + j); ids are k-digit base-K numbers (reading R21)."""
    L = lib()
    Pa = (ctypes.c_double * len(P))(*[float(x) for x in P])
    if len(P) != K * K:
        raise OracleError(-1, "kron_build_table: P must have K^2 entries")
    h = L.orc_table_new()
    rc = L.orc_kron_build_table(Pa, int(K), int(k), int(bound), int(mode), h)
    if rc != 0:
        L.orc_table_delete(h)
        raise OracleError(rc, "kron_build_table")
    return _wrap_table(h)


def _wrap_table(h) -> Table:
    L = lib()
    info = np.zeros(8, dtype=np.uint64)
    L.orc_table_info(h, _ptr(info))
    nb = int(info[5])
    arrs = dict(
        length=np.zeros(nb, np.uint8), code=np.zeros(nb, np.uint64), row=np.zeros(nb, np.uint32),
        col=np.zeros(nb, np.uint32), p=np.zeros(nb, np.float64), w=np.zeros(nb, np.int64),
        thr=np.zeros(nb, np.uint32), alias=np.zeros(nb, np.uint32))
    L.orc_table_arrays(h, *[_ptr(arrs[n]) for n in ("length", "code", "row", "col", "p", "w", "thr", "alias")])
    return Table(k=int(info[0]), mode=int(info[1]), cap=int(info[2]), bucket_bits=int(info[3]),
                 n_items=int(info[4]), n_buckets=nb, capacity=int(info[6]), handle=h, K=int(info[7]), **arrs)


UNDIRECTED = 1
SCRAMBLE = 2


def generate(t: Table, seed: int, edge_begin: int, m: int, threads: int = 1,
             width: int | None = None, samples: bool = False, flags: int = 0, scramble_key: int = 0):
    """Edges [edge_begin, edge_begin + m) as (src, dst[, samples per edge]).
    flags: UNDIRECTED (mirror to the upper triangle) and/or SCRAMBLE (relabel
    ids by the keyed bijection), Sec. 3 generalizations, reading R19."""
    if width is None:
        width = 4 if t.K ** t.k <= 2 ** 32 else 8
    dt = np.uint32 if width == 4 else np.uint64
    src = np.zeros(m, dt)
    dst = np.zeros(m, dt)
    ns = np.zeros(m, np.uint32) if samples else None
    rc = lib().orc_generate_ex(t.handle, seed, edge_begin, m, _ptr(src), _ptr(dst), width,
                               _ptr(ns) if samples else None, int(threads), int(flags), int(scramble_key))
    if rc != 0:
        raise OracleError(rc, "generate")
    return (src, dst, ns) if samples else (src, dst)


def generate_reduce(t: Table, seed: int, edge_begin: int, m: int, hist_bits: int = 16,
                    threads: int = 1):
    """Histogram of src >> (k - hist_bits) and XOR of edge_mix over the chunk."""
    hist = np.zeros(1 << hist_bits, np.uint64)
    x = np.zeros(1, np.uint64)
    rc = lib().orc_generate_reduce(t.handle, seed, edge_begin, m, hist_bits, _ptr(hist), _ptr(x), int(threads))
    if rc != 0:
        raise OracleError(rc, "generate_reduce")
    return hist, int(x[0])


# ---------------------------------------------------------------------------
# out-degrees: the workload's out-degree histogram read literally (one
# counter per node, reading R23), built from the edges of generate()

def out_degrees(t: Table, seed: int, edge_begin: int, m: int, threads: int = 8,
                slice_edges: int = 1 << 24) -> np.ndarray:
    """Out-degree of each of the 2^k nodes over edges [edge_begin, edge_begin + m):
    how many of those edges have it as source (uint64)."""
    if t.K != 2:
        raise OracleError(-1, "out_degrees (R-MAT tables only)")
    n = 1 << t.k
    deg = np.zeros(n, np.uint64)
    for off in range(0, m, slice_edges):
        src, _ = generate(t, seed, edge_begin + off, min(slice_edges, m - off), threads=threads)
        deg += np.bincount(src.astype(np.int64), minlength=n).astype(np.uint64)
    return deg


def degree_distribution(deg: np.ndarray, max_degree: int) -> np.ndarray:
    """Number of nodes of each out-degree 0 .. max_degree, the last bin counting
    every degree >= max_degree (uint64)."""
    clipped = np.minimum(deg.astype(np.uint64), np.uint64(max_degree)).astype(np.int64)
    return np.bincount(clipped, minlength=max_degree + 1).astype(np.uint64)


# ---------------------------------------------------------------------------
# partitioned generation (Sec. 3, reading R20)

def binomial(seed: int, r: int, c: int, level: int, n: int, p: float) -> int:
    """Bin(n, p) drawn from the uniform stream of tree node (level, r, c)."""
    return int(lib().orc_binomial(seed, r, c, level, n, p))


def partition_counts(t: Table, seed: int, m: int, tbits: int, row_begin: int = 0, row_end: int | None = None):
    """Edge counts of the 2^tbits x 2^tbits tiles in tile rows [row_begin,
    row_end), as a (rows, 2^tbits) uint64 array."""
    if row_end is None:
        row_end = 1 << tbits
    out = np.zeros(((row_end - row_begin), 1 << tbits), np.uint64)
    rc = lib().orc_partition_counts(t.handle, seed, m, tbits, row_begin, row_end, _ptr(out))
    if rc != 0:
        raise OracleError(rc, "partition_counts")
    return out


def generate_partition(t: Table, seed: int, m: int, tbits: int, row_begin: int = 0, row_end: int | None = None):
    """(counts, src, dst): the edges of the tiles in tile rows [row_begin,
    row_end), tile by tile in row-major order."""
    if row_end is None:
        row_end = 1 << tbits
    counts = partition_counts(t, seed, m, tbits, row_begin, row_end)
    n = int(counts.sum())
    dt = np.uint32 if t.k <= 32 else np.uint64
    src, dst = np.zeros(n, dt), np.zeros(n, dt)
    rc = lib().orc_generate_partition(t.handle, seed, m, tbits, row_begin, row_end, _ptr(src), _ptr(dst),
                                      4 if t.k <= 32 else 8, _ptr(counts))
    if rc != 0:
        raise OracleError(rc, "generate_partition")
    return counts, src, dst


# ---------------------------------------------------------------------------
# perturbed tables (Sec. 3, reading R22)

def perturbed_params(a, b, c, d, n_tables: int, eps: float, seed: int) -> np.ndarray:
    """(n_tables, 4) parameter sets: each entry scaled by 1 + eps (2u - 1),
    u from SplitMix64(seed), then normalised."""
    out = np.zeros((n_tables, 4), np.float64)
    rc = lib().orc_perturbed_params(a, b, c, d, n_tables, eps, seed, _ptr(out))
    if rc != 0:
        raise OracleError(rc, "perturbed_params")
    return out


def build_perturbed_tables(a, b, c, d, k, bound, mode, n_tables: int, eps: float, seed: int) -> list:
    return [build_table(*q, k, bound, mode) for q in perturbed_params(a, b, c, d, n_tables, eps, seed)]


def generate_set(tables: list, seed: int, edge_begin: int, m: int):
    """Edges [edge_begin, edge_begin + m), edge e from tables[e mod len(tables)]."""
    width = 4 if tables[0].k <= 32 else 8
    dt = np.uint32 if width == 4 else np.uint64
    src, dst = np.zeros(m, dt), np.zeros(m, dt)
    handles = (ctypes.c_void_p * len(tables))(*[t.handle for t in tables])
    rc = lib().orc_generate_set(handles, len(tables), seed, edge_begin, m, _ptr(src), _ptr(dst), width)
    if rc != 0:
        raise OracleError(rc, "generate_set")
    return src, dst
