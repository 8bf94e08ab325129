"""Device ceilings for the sampler's roofline (include/rmat_bench.h): HBM
write and copy bandwidth, Philox4x32-10 blocks per second, random 16-byte LDS
reads per second.  Each figure is the best of a few timed launches."""
from __future__ import annotations

import ctypes

from .rmat import _check, load


def _lib():
    L = load()
    if not hasattr(L, "_bench_ready"):
        vp, u64 = ctypes.c_void_p, ctypes.c_uint64
        L.rmat_bench_write.argtypes = [vp, u64, ctypes.c_int, vp]
        L.rmat_bench_copy.argtypes = [vp, vp, u64, vp]
        L.rmat_bench_philox.argtypes = [u64, ctypes.c_int, u64, vp, vp]
        L.rmat_bench_lds_read.argtypes = [u64, ctypes.c_uint32, ctypes.c_int, vp, vp]
        L.rmat_bench_gather.argtypes = [u64, vp, u64, ctypes.c_int, ctypes.c_int, vp, vp]
        L.rmat_bench_gather.restype = ctypes.c_int
        for n in ("rmat_bench_write", "rmat_bench_copy", "rmat_bench_philox", "rmat_bench_lds_read"):
            getattr(L, n).restype = ctypes.c_int
        L._bench_ready = True
    return L


def _time(fn, reps=5):
    import torch
    s = torch.cuda.current_stream()
    best = float("inf")
    fn(s)
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn(s)
        b.record(s)
        b.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    return best


def write_bandwidth(nbytes=8 << 30, vec_bytes=16) -> float:
    """GB/s of a store-only stream of nbytes."""
    import torch
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    L = _lib()
    t = _time(lambda s: _check(L.rmat_bench_write(buf.data_ptr(), nbytes, vec_bytes, s.cuda_stream),
                               "rmat_bench_write"))
    del buf
    return nbytes / t / 1e9


def copy_bandwidth(nbytes=4 << 30) -> float:
    """GB/s counting read + write bytes of a device-to-device copy."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    L = _lib()
    t = _time(lambda s: _check(L.rmat_bench_copy(a.data_ptr(), b.data_ptr(), nbytes, s.cuda_stream),
                               "rmat_bench_copy"))
    del a, b
    return 2 * nbytes / t / 1e9


def philox_rate(variant: int, n_blocks=1 << 32) -> float:
    """Philox4x32-10 blocks per second."""
    import torch
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    L = _lib()
    t = _time(lambda s: _check(L.rmat_bench_philox(n_blocks, variant, 0x1234, out.data_ptr(), s.cuda_stream),
                               "rmat_bench_philox"))
    return n_blocks / t


def philox_checksums(n_blocks=1 << 20):
    """XOR fold of the first n_blocks blocks for each variant (must agree)."""
    import torch
    L = _lib()
    res = []
    for v in range(3):
        out = torch.zeros(1, dtype=torch.int64, device="cuda")
        _check(L.rmat_bench_philox(n_blocks, v, 0x1234, out.data_ptr(), None), "rmat_bench_philox")
        torch.cuda.synchronize()
        res.append(int(out.item()) & (2**64 - 1))
    return res


def lds_read_rate(table_bytes=65536, width=16, n_reads=1 << 14) -> float:
    """Random LDS reads of `width` bytes per second over the whole device."""
    import torch
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    L = _lib()
    t = _time(lambda s: _check(L.rmat_bench_lds_read(n_reads, table_bytes, width, out.data_ptr(), s.cuda_stream),
                               "rmat_bench_lds_read"))
    threads = 256 * 4 * 512
    return threads * n_reads / t


def gather_rate(table_bytes=1 << 20, width=16, blocks_per_cu=2, n_reads=1 << 12) -> float:
    """Random reads of `width` bytes per second from a device table of
    table_bytes (L2-resident when it fits)."""
    import torch
    tab = torch.randint(0, 1 << 30, (table_bytes // 4,), dtype=torch.int32, device="cuda")
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    L = _lib()
    t = _time(lambda s: _check(L.rmat_bench_gather(n_reads, tab.data_ptr(), table_bytes, width, blocks_per_cu,
                                                   out.data_ptr(), s.cuda_stream), "rmat_bench_gather"))
    return 256 * blocks_per_cu * 512 * n_reads / t


def all_ceilings() -> dict:
    return {
        "write_gbs_16B": write_bandwidth(vec_bytes=16),
        "write_gbs_4B": write_bandwidth(vec_bytes=4),
        "copy_gbs": copy_bandwidth(),
        "philox_blocks_per_s": {f"v{v}": philox_rate(v) for v in range(3)},
        "lds_reads_per_s": {f"{w}B_{tb // 1024}KB": lds_read_rate(tb, w) for w in (4, 8, 16)
                            for tb in (16384, 65536)},
        "gather_reads_per_s": {f"{w}B_{tb >> 10}KB_x{bp}": gather_rate(tb, w, bp) for w in (4, 16)
                               for tb in (1 << 20, 1 << 16) for bp in (1, 2, 4)},
    }


if __name__ == "__main__":
    import json
    print(json.dumps(all_ceilings()))
