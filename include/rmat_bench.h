/*
 * rmat_bench.h -- microbenchmark kernels that measure the ceilings the R-MAT
 * sampler runs against on the device: streaming HBM writes, a plain copy
 * (the reference for HBM byte counters), Philox4x32-10 block throughput
 * (the per-edge random draw of the sampler) and random 16-byte LDS reads
 * (the per-sample alias-table lookup).  None of them is part of the method;
 * they exist to put the sampler's measured rate next to what the hardware
 * allows.  All are asynchronous on `stream` (a hipStream_t, NULL for the
 * null stream), take device pointers owned by the caller, and return an
 * rmat_status (include/rmat.h) with rmat_last_error() set on failure.
 */
#ifndef RMAT_BENCH_H
#define RMAT_BENCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Writes `bytes` (a multiple of 16) to d_dst with coalesced stores of
 * `vec_bytes` (4, 8 or 16) per lane; no reads.  RMAT_EINVAL on bad sizes. */
int rmat_bench_write(void* d_dst, uint64_t bytes, int vec_bytes, void* stream);

/* Copies `bytes` (a multiple of 16) from d_src to d_dst with 16-byte loads
 * and stores.  Used to calibrate HBM byte counters against a known size. */
int rmat_bench_copy(const void* d_src, void* d_dst, uint64_t bytes, void* stream);

/* Computes n_blocks Philox4x32-10 blocks (key = seed, counter = (i, 0, 0, 0))
 * and XOR-folds them into d_out[0] (uint64).  variant 0: 32-bit mul_lo/mul_hi
 * and two-input XORs; 1: one 32x32->64 multiply-add per product and
 * three-input XORs; 2: variant 1 with the first two rounds simplified for a
 * zero high counter word.  All variants produce the same value. */
int rmat_bench_philox(uint64_t n_blocks, int variant, uint64_t seed, void* d_out, void* stream);

/* Performs n_reads (a multiple of 8) random LDS reads of `width` bytes (4, 8
 * or 16) per lane, from a table of table_bytes (a power of two, 16 .. 65536),
 * in 512-lane workgroups with 8 independent address streams per lane, and
 * XOR-folds the data into d_out[0]. */
int rmat_bench_lds_read(uint64_t n_reads, uint32_t table_bytes, int width, void* d_out, void* stream);

/* Performs n_reads (a multiple of 8) random reads of `width` bytes (4, 8 or
 * 16) per lane from the device table d_table of table_bytes (a power of two;
 * one of L2 size stays in L2), in 256 * blocks_per_cu (1..4) workgroups of
 * 512 lanes with 8 independent address streams per lane, and XOR-folds the
 * data into d_out[0]: the random-gather ceiling of a table read from L2. */
int rmat_bench_gather(uint64_t n_reads, const void* d_table, uint64_t table_bytes, int width, int blocks_per_cu,
                      void* d_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RMAT_BENCH_H */
