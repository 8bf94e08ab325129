"""Profiling target: one build + one generation of the benchmark instance
(k = 26, 2^30 edges, 4096-entry variable table, a=0.57 b=c=0.19 d=0.05,
seed 7), then one plain 1 GiB device copy whose HBM traffic is known (read
1 GiB, write 1 GiB), to scale the hardware byte counters.

    rocprofv3 --kernel-trace --stats -d OUT -- python3 -m paper_1905_03525_amd.profile_target
    rocprofv3 --pmc FETCH_SIZE -d OUT -- python3 -m paper_1905_03525_amd.profile_target
"""
from __future__ import annotations

import argparse
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=1, help="generations of the instance")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--lds-bench", action="store_true",
                    help="also run the random LDS read microbenchmark (16-, 8- and 4-byte reads)")
    args = ap.parse_args()
    import torch

    from . import rmat as R
    from .microbench import _lib

    torch.cuda.set_device(0)
    m, k = 1 << 30, 26
    src = torch.empty(m, dtype=torch.int32, device="cuda")
    dst = torch.empty(m, dtype=torch.int32, device="cuda")
    t = R.rmat_build_table(0.57, 0.19, 0.19, 0.05, k, 4096, R.RMAT_VARIABLE)
    print("table built", flush=True)
    for _ in range(args.reps):
        R.rmat_generate(t, 7, 0, m, src, dst)
    print(f"generated {args.reps} x {m} edges", flush=True)
    a = torch.empty(args.copy_bytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(args.copy_bytes, dtype=torch.uint8, device="cuda")
    R._check(_lib().rmat_bench_copy(a.data_ptr(), b.data_ptr(), args.copy_bytes, None), "rmat_bench_copy")
    torch.cuda.synchronize()
    print(f"copied {args.copy_bytes} bytes", flush=True)
    if args.lds_bench:
        out = torch.zeros(1, dtype=torch.int64, device="cuda")
        for width in (16, 8, 4):
            R._check(_lib().rmat_bench_lds_read(1 << 12, 65536, width, out.data_ptr(), None), "rmat_bench_lds_read")
        torch.cuda.synchronize()
        print("lds microbenchmarks done", flush=True)
    t.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
