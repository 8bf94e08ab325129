"""Writes k34_chunk_digests.txt: the oracle's reduction of each 2^30-edge
chunk of the k = 34, m = 2^34 instance (a, b, c, d = 0.45, 0.22, 0.22, 0.11,
variable-length table bounded at 2^16 paths, Philox seed 3): the SHA-256 of
the 2^16-bin source-prefix histogram (little-endian uint64 counts), its total,
and the XOR checksum.  Calls only the oracle.

    python tests/golden/make_k34_chunk_digests.py [threads]
"""
import hashlib
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402

Q, K, BOUND, SEED, CHUNK, N_CHUNKS, HIST_BITS = (0.45, 0.22, 0.22, 0.11), 34, 1 << 16, 3, 1 << 30, 16, 16


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    t = oracle.build_table(*Q, K, BOUND, oracle.VARIABLE)
    lines = ["# oracle reduction of the k=34, m=2^34 instance in 2^30-edge chunks",
             f"# a,b,c,d={Q} k={K} bound={BOUND} variable seed={SEED} hist_bits={HIST_BITS}",
             "# chunk edge_begin m hist_sha256 hist_total xor_hex"]
    for c in range(N_CHUNKS):
        t0 = time.time()
        hist, x = oracle.generate_reduce(t, SEED, c * CHUNK, CHUNK, hist_bits=HIST_BITS, threads=threads)
        h = hashlib.sha256(hist.astype("<u8").tobytes()).hexdigest()
        lines.append(f"{c} {c * CHUNK} {CHUNK} {h} {int(hist.sum())} {x:016x}")
        print(lines[-1], f"({time.time() - t0:.1f} s)", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "k34_chunk_digests.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
