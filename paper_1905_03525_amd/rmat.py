"""ctypes binding of librmat.so: the C ABI of include/rmat.h under the same
names.  Argument marshalling only; every step runs in the HIP library.  torch
supplies device memory and streams.  Importing this module loads nothing;
the first call loads librmat.so and raises if it is missing (there is no
fallback)."""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librmat.so")

RMAT_FIXED = 0
RMAT_VARIABLE = 1
RMAT_UNDIRECTED = 1
RMAT_SCRAMBLE = 2

RMAT_OK = 0
RMAT_EINVAL = -1
RMAT_ENOMEM = -2
RMAT_EDEVICE = -3
RMAT_ERANGE = -4
_STATUS = {RMAT_EINVAL: "RMAT_EINVAL", RMAT_ENOMEM: "RMAT_ENOMEM", RMAT_EDEVICE: "RMAT_EDEVICE",
           RMAT_ERANGE: "RMAT_ERANGE"}

# Every symbol include/rmat.h declares (checked by the CPU test suite).
EXPORTED = ["rmat_build_table", "rmat_build_table_async", "rmat_kron_build_table", "rmat_build_perturbed_table", "rmat_table_export_member", "rmat_free_table", "rmat_table_info", "rmat_table_export", "rmat_generate",
            "rmat_generate_async", "rmat_generate_ex_async", "rmat_generate_reduce_async",
            "rmat_generate_reduce_noalloc_async", "rmat_generate_degrees_async",
            "rmat_degree_distribution_async", "rmat_batch_create", "rmat_batch_enqueue",
            "rmat_partition_counts", "rmat_generate_partition", "rmat_generate_partition_async", "rmat_batch_launch_graph", "rmat_batch_check", "rmat_batch_table_info", "rmat_batch_table_export", "rmat_batch_get_info",
            "rmat_batch_free", "rmat_batch_autotune", "rmat_server_create", "rmat_server_submit",
            "rmat_server_step", "rmat_server_drain", "rmat_server_poll", "rmat_server_release",
            "rmat_server_run_trace", "rmat_server_get_stats", "rmat_server_clock", "rmat_server_free",
            "rmat_last_error"]
RMAT_REQ_DIGEST = 1
RMAT_REQ_DISCARD = 2
RMAT_REQ_UNDIRECTED = 4
RMAT_REQ_SCRAMBLE = 8


class RmatError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


class rmat_info(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("path_mode", ctypes.c_int32), ("depth_cap", ctypes.c_int32),
                ("bucket_bits", ctypes.c_int32), ("table_bound", ctypes.c_uint64), ("n_items", ctypes.c_uint64),
                ("n_buckets", ctypes.c_uint64), ("capacity", ctypes.c_uint64), ("id_bytes", ctypes.c_uint32),
                ("min_len", ctypes.c_uint32), ("max_len", ctypes.c_uint32), ("lds_resident", ctypes.c_uint32),
                ("expected_len", ctypes.c_double), ("export_bytes", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("initiator_k", ctypes.c_uint32), ("n_tables", ctypes.c_uint32)]


class rmat_instance(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("c", ctypes.c_double), ("d", ctypes.c_double),
                ("k", ctypes.c_int32), ("path_mode", ctypes.c_int32), ("table_bound", ctypes.c_uint64),
                ("seed", ctypes.c_uint64), ("edge_begin", ctypes.c_uint64), ("m", ctypes.c_uint64),
                ("out_src", ctypes.c_void_p), ("out_dst", ctypes.c_void_p), ("flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("scramble_key", ctypes.c_uint64)]


class rmat_batch_info(ctypes.Structure):
    _fields_ = [("n_instances", ctypes.c_uint32), ("n_launches", ctypes.c_uint32),
                ("n_work_items", ctypes.c_uint32), ("work_blocks", ctypes.c_uint32),
                ("tile_blocks", ctypes.c_uint32), ("max_buckets", ctypes.c_uint32),
                ("total_edges", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64)]


class rmat_autotune_report(ctypes.Structure):
    _fields_ = [("search_seconds", ctypes.c_double), ("calibration_ns", ctypes.c_double),
                ("n_tuned", ctypes.c_uint32), ("n_candidates", ctypes.c_uint32),
                ("work_blocks", ctypes.c_uint32), ("chosen", ctypes.c_uint32), ("measured", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("model_ms", ctypes.c_double), ("tuned_ms", ctypes.c_double),
                ("all_4096_ms", ctypes.c_double), ("all_8192_ms", ctypes.c_double)]


class rmat_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_table_bound", ctypes.c_uint64),
                ("tick_blocks", ctypes.c_uint64), ("request_quantum", ctypes.c_uint64),
                ("max_active", ctypes.c_uint32), ("table_slots", ctypes.c_uint32), ("work_blocks", ctypes.c_uint32),
                ("max_inflight", ctypes.c_uint32), ("max_builds", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class rmat_request(ctypes.Structure):
    _fields_ = [("a", ctypes.c_double), ("b", ctypes.c_double), ("c", ctypes.c_double), ("d", ctypes.c_double),
                ("k", ctypes.c_int32), ("path_mode", ctypes.c_int32), ("table_bound", ctypes.c_uint64),
                ("seed", ctypes.c_uint64), ("edge_begin", ctypes.c_uint64), ("m", ctypes.c_uint64),
                ("out_src", ctypes.c_void_p), ("out_dst", ctypes.c_void_p), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32), ("scramble_key", ctypes.c_uint64)]


class rmat_completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("table_hit", ctypes.c_uint32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("digest", ctypes.c_uint64), ("out_src", ctypes.c_void_p), ("out_dst", ctypes.c_void_p)]


class rmat_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("rounds", ctypes.c_uint64), ("table_builds", ctypes.c_uint64),
                ("table_hits", ctypes.c_uint64), ("edges_done", ctypes.c_uint64), ("arena_bytes", ctypes.c_uint64),
                ("arena_peak", ctypes.c_uint64), ("active", ctypes.c_uint32), ("pending", ctypes.c_uint32),
                ("device_bytes", ctypes.c_uint64)]


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64)

_lib = None


def load() -> ctypes.CDLL:
    """Loads librmat.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1905_03525_amd.build "
                           "(there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, c_int = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int
    L.rmat_build_table.argtypes = [ctypes.c_double] * 4 + [c_int, u64, c_int, ctypes.POINTER(vp)]
    L.rmat_build_table_async.argtypes = [ctypes.c_double] * 4 + [c_int, u64, c_int, vp, ctypes.POINTER(vp)]
    L.rmat_free_table.argtypes = [vp]
    L.rmat_build_perturbed_table.argtypes = [ctypes.c_double] * 4 + [c_int, u64, c_int, c_int, ctypes.c_double, u64,
                                                                      ctypes.POINTER(vp)]
    L.rmat_table_export_member.argtypes = [vp, c_int, vp, ctypes.c_size_t]
    L.rmat_kron_build_table.argtypes = [ctypes.POINTER(ctypes.c_double), c_int, c_int, u64, c_int,
                                        ctypes.POINTER(vp)]
    L.rmat_table_info.argtypes = [vp, ctypes.POINTER(rmat_info)]
    L.rmat_table_export.argtypes = [vp, vp, ctypes.c_size_t]
    L.rmat_generate.argtypes = [vp, u64, u64, u64, vp, vp]
    L.rmat_generate_async.argtypes = [vp, u64, u64, u64, vp, vp, vp]
    L.rmat_generate_reduce_async.argtypes = [vp, u64, u64, u64, c_int, vp, vp, vp]
    L.rmat_generate_reduce_noalloc_async.argtypes = [vp, u64, u64, u64, c_int, vp, vp, vp]
    L.rmat_generate_ex_async.argtypes = [vp, u64, u64, u64, c_int, u64, vp, vp, vp]
    L.rmat_generate_degrees_async.argtypes = [vp, u64, u64, u64, vp, vp]
    L.rmat_degree_distribution_async.argtypes = [vp, u64, ctypes.c_uint32, vp, vp]
    L.rmat_partition_counts.argtypes = [vp, u64, u64, c_int, ctypes.c_uint32, ctypes.c_uint32, vp]
    L.rmat_generate_partition.argtypes = [vp, u64, u64, c_int, ctypes.c_uint32, ctypes.c_uint32, vp, vp, u64]
    L.rmat_generate_partition_async.argtypes = [vp, u64, u64, c_int, ctypes.c_uint32, ctypes.c_uint32, vp, vp, u64,
                                                vp]
    L.rmat_batch_create.argtypes = [ctypes.POINTER(rmat_instance), c_int, ctypes.c_uint32, ctypes.POINTER(vp)]
    L.rmat_batch_enqueue.argtypes = [vp, vp]
    L.rmat_batch_launch_graph.argtypes = [vp, vp]
    L.rmat_batch_check.argtypes = [vp]
    L.rmat_batch_table_info.argtypes = [vp, c_int, ctypes.POINTER(rmat_info)]
    L.rmat_batch_table_export.argtypes = [vp, c_int, vp, ctypes.c_size_t]
    L.rmat_batch_get_info.argtypes = [vp, ctypes.POINTER(rmat_batch_info)]
    L.rmat_batch_free.argtypes = [vp]
    L.rmat_batch_autotune.argtypes = [ctypes.POINTER(rmat_instance), c_int, ctypes.POINTER(rmat_autotune_report)]
    L.rmat_server_create.argtypes = [ctypes.POINTER(rmat_server_config), ctypes.POINTER(vp)]
    L.rmat_server_submit.argtypes = [vp, ctypes.POINTER(rmat_request), ctypes.c_double, ctypes.POINTER(u64)]
    L.rmat_server_step.argtypes = [vp, ctypes.POINTER(c_int)]
    L.rmat_server_drain.argtypes = [vp]
    L.rmat_server_poll.argtypes = [vp, ctypes.POINTER(rmat_completion), c_int, ctypes.POINTER(c_int)]
    L.rmat_server_release.argtypes = [vp, u64]
    L.rmat_server_run_trace.argtypes = [vp, ctypes.POINTER(rmat_request), ctypes.POINTER(ctypes.c_double), c_int,
                                        ctypes.POINTER(rmat_completion), PROGRESS_FN, vp]
    L.rmat_server_get_stats.argtypes = [vp, ctypes.POINTER(rmat_server_stats)]
    L.rmat_server_clock.argtypes = [vp]
    L.rmat_server_free.argtypes = [vp]
    L.rmat_last_error.argtypes = []
    L.rmat_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name != "rmat_last_error":
            getattr(L, name).restype = c_int
    L.rmat_server_clock.restype = ctypes.c_double
    _lib = L
    return L


def _check(status: int, func: str):
    if status != RMAT_OK:
        raise RmatError(status, func, load().rmat_last_error().decode())


def _ptr(x) -> int | None:
    """Device pointer of a torch tensor, or an int address, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s) -> int | None:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


class Table:
    """Owning handle of an rmat_table_t."""

    def __init__(self, handle: int):
        self.handle = handle

    def close(self):
        if self.handle:
            _check(load().rmat_free_table(self.handle), "rmat_free_table")
            self.handle = None

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rmat_free_table(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def rmat_build_table(a: float, b: float, c: float, d: float, k: int, table_bound: int, path_mode: int) -> Table:
    h = ctypes.c_void_p()
    _check(load().rmat_build_table(a, b, c, d, k, table_bound, path_mode, ctypes.byref(h)), "rmat_build_table")
    return Table(h.value)


def rmat_build_table_async(a: float, b: float, c: float, d: float, k: int, table_bound: int, path_mode: int,
                           stream=None) -> Table:
    h = ctypes.c_void_p()
    _check(load().rmat_build_table_async(a, b, c, d, k, table_bound, path_mode, _stream(stream), ctypes.byref(h)),
           "rmat_build_table_async")
    return Table(h.value)


def rmat_kron_build_table(P, K: int, k: int, table_bound: int, path_mode: int) -> Table:
    """Table of a K x K Kronecker initiator P (K^2 probabilities, row-major)."""
    arr = (ctypes.c_double * len(P))(*[float(x) for x in P])
    h = ctypes.c_void_p()
    _check(load().rmat_kron_build_table(arr, K, k, table_bound, path_mode, ctypes.byref(h)), "rmat_kron_build_table")
    return Table(h.value)


def rmat_build_perturbed_table(a, b, c, d, k, table_bound, path_mode, n_tables, epsilon, perturb_seed) -> Table:
    h = ctypes.c_void_p()
    _check(load().rmat_build_perturbed_table(a, b, c, d, k, table_bound, path_mode, n_tables, epsilon, perturb_seed,
                                             ctypes.byref(h)), "rmat_build_perturbed_table")
    return Table(h.value)


def rmat_table_export_member(t: Table, i: int) -> dict:
    info = rmat_table_info(t)
    buf = np.zeros(info["export_bytes"], dtype=np.uint8)
    _check(load().rmat_table_export_member(t.handle, i, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes),
           "rmat_table_export_member")
    return _split_export(buf, info["n_buckets"])


def rmat_free_table(t: Table):
    t.close()


def rmat_table_info(t: Table) -> dict:
    info = rmat_info()
    _check(load().rmat_table_info(t.handle, ctypes.byref(info)), "rmat_table_info")
    return {name: getattr(info, name) for name, _ in rmat_info._fields_}


def _split_export(buf: np.ndarray, nb: int) -> dict:
    out, off = {}, 0
    for name, dt in (("w", np.uint64), ("p", np.float64), ("len", np.uint32), ("row", np.uint32),
                     ("col", np.uint32), ("thr", np.uint32), ("alias", np.uint32)):
        n = nb * np.dtype(dt).itemsize
        out[name] = buf[off:off + n].view(dt).copy()
        off += n
    return out


def rmat_table_export(t: Table) -> dict:
    """Canonical table arrays (see include/rmat.h) as numpy arrays."""
    info = rmat_table_info(t)
    nb = info["n_buckets"]
    buf = np.zeros(info["export_bytes"], dtype=np.uint8)
    _check(load().rmat_table_export(t.handle, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes), "rmat_table_export")
    return _split_export(buf, nb)


def rmat_generate(t: Table, seed: int, edge_begin: int, m: int, out_src, out_dst):
    _check(load().rmat_generate(t.handle, seed, edge_begin, m, _ptr(out_src), _ptr(out_dst)), "rmat_generate")


def rmat_generate_async(t: Table, seed: int, edge_begin: int, m: int, out_src, out_dst, stream=None):
    _check(load().rmat_generate_async(t.handle, seed, edge_begin, m, _ptr(out_src), _ptr(out_dst),
                                      _stream(stream)), "rmat_generate_async")


def rmat_generate_ex_async(t: Table, seed: int, edge_begin: int, m: int, flags: int, scramble_key: int, out_src,
                           out_dst, stream=None):
    _check(load().rmat_generate_ex_async(t.handle, seed, edge_begin, m, flags, scramble_key, _ptr(out_src),
                                         _ptr(out_dst), _stream(stream)), "rmat_generate_ex_async")


def rmat_partition_counts(t: Table, seed: int, m: int, tile_bits: int, row_begin: int = 0,
                          row_end: int | None = None) -> np.ndarray:
    """Edge counts of the tiles in tile rows [row_begin, row_end), shape (rows, 2^tile_bits)."""
    if row_end is None:
        row_end = 1 << tile_bits
    out = np.zeros((row_end - row_begin, 1 << tile_bits), np.uint64)
    _check(load().rmat_partition_counts(t.handle, seed, m, tile_bits, row_begin, row_end,
                                        out.ctypes.data_as(ctypes.c_void_p)), "rmat_partition_counts")
    return out


def rmat_generate_partition(t: Table, seed: int, m: int, tile_bits: int, row_begin: int, row_end: int, out_src,
                            out_dst, n_out: int):
    _check(load().rmat_generate_partition(t.handle, seed, m, tile_bits, row_begin, row_end, _ptr(out_src),
                                          _ptr(out_dst), n_out), "rmat_generate_partition")


def rmat_generate_partition_async(t: Table, seed: int, m: int, tile_bits: int, row_begin: int, row_end: int,
                                  out_src, out_dst, n_out: int, stream=None):
    _check(load().rmat_generate_partition_async(t.handle, seed, m, tile_bits, row_begin, row_end, _ptr(out_src),
                                                _ptr(out_dst), n_out, _stream(stream)),
           "rmat_generate_partition_async")


def generate_partition(t: Table, seed: int, m: int, tile_bits: int, row_begin: int = 0, row_end: int | None = None,
                       device="cuda"):
    """(counts, src, dst) of the tiles in tile rows [row_begin, row_end); the
    outputs are allocated on the device."""
    import torch
    counts = rmat_partition_counts(t, seed, m, tile_bits, row_begin, row_end)
    n = int(counts.sum())
    k = rmat_table_info(t)["k"]
    src = torch.empty(max(n, 1), dtype=id_dtype(k), device=device)
    dst = torch.empty(max(n, 1), dtype=id_dtype(k), device=device)
    rmat_generate_partition(t, seed, m, tile_bits, row_begin, row_end if row_end is not None else 1 << tile_bits,
                            src, dst, n)
    return counts, src[:n], dst[:n]


def rmat_generate_reduce_async(t: Table, seed: int, edge_begin: int, m: int, hist_bits: int, d_hist, d_xor,
                               stream=None):
    _check(load().rmat_generate_reduce_async(t.handle, seed, edge_begin, m, hist_bits, _ptr(d_hist), _ptr(d_xor),
                                             _stream(stream)), "rmat_generate_reduce_async")


def rmat_generate_reduce_noalloc_async(t: Table, seed: int, edge_begin: int, m: int, hist_bits: int, d_hist, d_xor,
                                       stream=None):
    _check(load().rmat_generate_reduce_noalloc_async(t.handle, seed, edge_begin, m, hist_bits, _ptr(d_hist),
                                                     _ptr(d_xor), _stream(stream)), "rmat_generate_reduce_noalloc_async")


def rmat_generate_degrees_async(t: Table, seed: int, edge_begin: int, m: int, d_degree, stream=None):
    """d_degree[src] += 1 for every edge of [edge_begin, edge_begin + m)
    (2^k uint32 counters on the device)."""
    _check(load().rmat_generate_degrees_async(t.handle, seed, edge_begin, m, _ptr(d_degree), _stream(stream)),
           "rmat_generate_degrees_async")


def rmat_degree_distribution_async(d_degree, n_nodes: int, max_degree: int, d_hist, stream=None):
    """d_hist[min(d, max_degree)] += 1 for each of n_nodes uint32 counters d."""
    _check(load().rmat_degree_distribution_async(_ptr(d_degree), n_nodes, max_degree, _ptr(d_hist),
                                                 _stream(stream)), "rmat_degree_distribution_async")


def rmat_last_error() -> str:
    return load().rmat_last_error().decode()


def id_dtype(k: int, id_bytes: int | None = None):
    """torch dtype holding the ids of a table with this k (bit patterns);
    id_bytes overrides (Kronecker tables: 4 if K^k <= 2^32)."""
    import torch
    if id_bytes is not None:
        return torch.int32 if id_bytes == 4 else torch.int64
    return torch.int32 if k <= 32 else torch.int64


def to_numpy_ids(x, k: int) -> np.ndarray:
    """Device id tensor -> numpy array of uint32 / uint64 (by the tensor's width)."""
    a = x.cpu().numpy()
    return a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint64)


def generate_edges(t: Table, seed: int, edge_begin: int, m: int, device="cuda", stream=None):
    """Allocates (src, dst) on the device and enqueues rmat_generate_async on
    `stream` (default: torch's current stream)."""
    import torch
    info = rmat_table_info(t)
    src = torch.empty(m, dtype=id_dtype(info["k"], info["id_bytes"]), device=device)
    dst = torch.empty(m, dtype=id_dtype(info["k"], info["id_bytes"]), device=device)
    if stream is None:
        stream = torch.cuda.current_stream(src.device)
    rmat_generate_async(t, seed, edge_begin, m, src, dst, stream)
    return src, dst


# ---------------------------------------------------------------------------
# batches

def make_instances(params) -> "ctypes.Array":
    """Array of rmat_instance from dicts with keys a, b, c, d, k, path_mode,
    table_bound, seed, edge_begin, m, out_src, out_dst (tensors or ints)."""
    arr = (rmat_instance * len(params))()
    for x, p in zip(arr, params):
        x.a, x.b, x.c, x.d = p["a"], p["b"], p["c"], p["d"]
        x.k, x.path_mode = p["k"], p.get("path_mode", RMAT_VARIABLE)
        x.table_bound, x.seed = p.get("table_bound", 0), p["seed"]
        x.edge_begin, x.m = p.get("edge_begin", 0), p["m"]
        x.out_src, x.out_dst = _ptr(p.get("out_src")), _ptr(p.get("out_dst"))
        x.flags, x.scramble_key = p.get("gen_flags", 0), p.get("scramble_key", 0)
    return arr


class Batch:
    """Owning handle of an rmat_batch_t."""

    def __init__(self, handle: int, n: int):
        self.handle = handle
        self.n = n

    def close(self):
        if self.handle:
            _check(load().rmat_batch_free(self.handle), "rmat_batch_free")
            self.handle = None

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rmat_batch_free(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def rmat_batch_create(instances, work_blocks: int = 0) -> Batch:
    """instances: an rmat_instance array (make_instances) or a list of dicts."""
    arr = instances if isinstance(instances, ctypes.Array) else make_instances(instances)
    h = ctypes.c_void_p()
    _check(load().rmat_batch_create(arr, len(arr), work_blocks, ctypes.byref(h)), "rmat_batch_create")
    return Batch(h.value, len(arr))


def rmat_batch_enqueue(b: Batch, stream=None):
    _check(load().rmat_batch_enqueue(b.handle, _stream(stream)), "rmat_batch_enqueue")


def rmat_batch_launch_graph(b: Batch, stream=None):
    _check(load().rmat_batch_launch_graph(b.handle, _stream(stream)), "rmat_batch_launch_graph")


def rmat_batch_check(b: Batch):
    _check(load().rmat_batch_check(b.handle), "rmat_batch_check")


def rmat_batch_get_info(b: Batch) -> dict:
    info = rmat_batch_info()
    _check(load().rmat_batch_get_info(b.handle, ctypes.byref(info)), "rmat_batch_get_info")
    return {name: getattr(info, name) for name, _ in rmat_batch_info._fields_}


def rmat_batch_table_info(b: Batch, i: int) -> dict:
    info = rmat_info()
    _check(load().rmat_batch_table_info(b.handle, i, ctypes.byref(info)), "rmat_batch_table_info")
    return {name: getattr(info, name) for name, _ in rmat_info._fields_}


def rmat_batch_table_export(b: Batch, i: int) -> dict:
    n_buckets = rmat_batch_table_info(b, i)["n_buckets"]
    buf = np.zeros(36 * n_buckets, dtype=np.uint8)
    _check(load().rmat_batch_table_export(b.handle, i, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes),
           "rmat_batch_table_export")
    return _split_export(buf, n_buckets)


def rmat_batch_free(b: Batch):
    b.close()


def rmat_batch_autotune(instances) -> dict:
    """Fills table_bound in place for entries that hold 0 (an rmat_instance
    array; a list of dicts is updated too) and returns the report."""
    arr = instances if isinstance(instances, ctypes.Array) else make_instances(instances)
    rep = rmat_autotune_report()
    _check(load().rmat_batch_autotune(arr, len(arr), ctypes.byref(rep)), "rmat_batch_autotune")
    if not isinstance(instances, ctypes.Array):
        for p, x in zip(instances, arr):
            p["table_bound"] = x.table_bound
    return {name: getattr(rep, name) for name, _ in rmat_autotune_report._fields_}


# ---------------------------------------------------------------------------
# request server

def _struct_dict(x) -> dict:
    return {name: getattr(x, name) for name, _ in x._fields_}


def make_request(p: dict) -> rmat_request:
    r = rmat_request()
    r.a, r.b, r.c, r.d = p["a"], p["b"], p["c"], p["d"]
    r.k, r.path_mode = p["k"], p.get("path_mode", RMAT_VARIABLE)
    r.table_bound, r.seed = p["table_bound"], p["seed"]
    r.edge_begin, r.m = p.get("edge_begin", 0), p["m"]
    r.out_src, r.out_dst = _ptr(p.get("out_src")), _ptr(p.get("out_dst"))
    r.flags = p.get("flags", 0)
    r.scramble_key = p.get("scramble_key", 0)
    return r


class Server:
    """Owning handle of an rmat_server_t."""

    def __init__(self, handle: int):
        self.handle = handle

    def close(self):
        if self.handle:
            _check(load().rmat_server_free(self.handle), "rmat_server_free")
            self.handle = None

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rmat_server_free(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def rmat_server_create(**cfg) -> Server:
    """Keyword arguments are rmat_server_config fields (0 / absent: default)."""
    c = rmat_server_config()
    for key, val in cfg.items():
        setattr(c, key, val)
    h = ctypes.c_void_p()
    _check(load().rmat_server_create(ctypes.byref(c), ctypes.byref(h)), "rmat_server_create")
    return Server(h.value)


def rmat_server_submit(s: Server, p: dict, t_arrival: float = -1.0) -> int:
    r = make_request(p)
    t = ctypes.c_uint64()
    _check(load().rmat_server_submit(s.handle, ctypes.byref(r), t_arrival, ctypes.byref(t)), "rmat_server_submit")
    return t.value


def rmat_server_step(s: Server) -> bool:
    busy = ctypes.c_int()
    _check(load().rmat_server_step(s.handle, ctypes.byref(busy)), "rmat_server_step")
    return bool(busy.value)


def rmat_server_drain(s: Server):
    _check(load().rmat_server_drain(s.handle), "rmat_server_drain")


def rmat_server_poll(s: Server, max_n: int = 4096) -> list:
    buf = (rmat_completion * max_n)()
    n = ctypes.c_int()
    _check(load().rmat_server_poll(s.handle, buf, max_n, ctypes.byref(n)), "rmat_server_poll")
    return [_struct_dict(buf[i]) for i in range(n.value)]


def rmat_server_release(s: Server, ticket: int):
    _check(load().rmat_server_release(s.handle, ticket), "rmat_server_release")


def rmat_server_run_trace(s: Server, requests: list, t_arrival, progress=None) -> list:
    """Serves `requests` (dicts) arriving at t_arrival (seconds, ascending);
    returns one completion dict per request, in request order.  progress, if
    given, is called as progress(done, total) about once a second."""
    n = len(requests)
    arr = (rmat_request * n)(*[make_request(p) for p in requests])
    ts = (ctypes.c_double * n)(*[float(t) for t in t_arrival])
    out = (rmat_completion * n)()
    cb = PROGRESS_FN(lambda _u, done, total: progress(done, total)) if progress else PROGRESS_FN()
    _check(load().rmat_server_run_trace(s.handle, arr, ts, n, out, cb, None), "rmat_server_run_trace")
    return [_struct_dict(out[i]) for i in range(n)]


def rmat_server_get_stats(s: Server) -> dict:
    st = rmat_server_stats()
    _check(load().rmat_server_get_stats(s.handle, ctypes.byref(st)), "rmat_server_get_stats")
    return _struct_dict(st)


def rmat_server_clock(s: Server) -> float:
    return load().rmat_server_clock(s.handle)


def rmat_server_free(s: Server):
    s.close()
