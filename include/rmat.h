/*
 * rmat.h -- C ABI of the MI355X (gfx950) linear-work R-MAT edge sampler.
 *
 * Method: Huebschle-Schneider & Sanders, "Linear Work Generation of R-MAT
 * Graphs" (arXiv 1905.03525).  Sec. 1 defines the R-MAT process: a directed
 * multigraph with n = 2^k nodes and m edges; each edge descends k times into
 * one of the four quadrants of the adjacency matrix, upper left with
 * probability a, upper right b, lower left c, lower right d (a+b+c+d = 1),
 * fixing one row bit and one column bit per level.  Sec. 2 precomputes a
 * table of quadrant paths with their probabilities (all paths of one length,
 * or the variable-length set grown by a max-priority queue that always
 * expands the most probable path), samples paths from it in constant time
 * with a Walker alias structure, and concatenates their row/column bits until
 * k bits are known.
 *
 * Conventions shared by every entry point:
 *  - Letters: a = (row 0, col 0), b = (0, 1), c = (1, 0), d = (1, 1).  The
 *    row id is the source, the column id the destination.  The root-most
 *    letter is the most significant id bit.
 *  - Ids are uint32 when k <= 32 and uint64 when k > 32.  Edge e of the
 *    global stream goes to slot e - edge_begin of the output arrays.
 *  - Randomness: Philox4x32-10 (Salmon et al., SC'11), key (seed_lo,
 *    seed_hi), counter (e_lo, e_hi, j, 0); sample s of edge e is word s mod 4
 *    of counter j = s / 4.  Each edge owns its counter stream, so any split
 *    of [0, m) into calls produces the same edges, and letters left after
 *    the k-th are discarded (the paper carries them to the next edge).
 *  - Device pointers are HIP device addresses on the current device and are
 *    owned by the caller.  Host pointers are plain host memory.
 *  - Every function returns an rmat_status; none throws or aborts.  On error
 *    rmat_last_error() returns a thread-local message and outputs are left
 *    untouched (generation errors detected after a launch may have written
 *    part of the output).
 */
#ifndef RMAT_H
#define RMAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rmat_table* rmat_table_t;

/* Path sets of Sec. 2. */
enum rmat_path_mode {
  RMAT_FIXED = 0,    /* all 4^l paths of length l = floor(log4 bound) */
  RMAT_VARIABLE = 1  /* priority-queue expansion, 1 + 3 ceil((bound-4)/3) paths */
};

enum rmat_status {
  RMAT_OK = 0,
  RMAT_EINVAL = -1,   /* invalid argument */
  RMAT_ENOMEM = -2,   /* device or host allocation failed */
  RMAT_EDEVICE = -3,  /* HIP runtime error or no usable gfx950 device */
  RMAT_ERANGE = -4    /* edge_begin + m overflows 2^64 */
};

typedef struct rmat_info {
  int32_t k;
  int32_t path_mode;
  int32_t depth_cap;       /* min(15, k): longest path in the table */
  int32_t bucket_bits;     /* b: the alias table has 2^b buckets */
  uint64_t table_bound;
  uint64_t n_items;        /* |A|, number of paths */
  uint64_t n_buckets;      /* 2^b; items n_items..2^b-1 are zero-weight padding */
  uint64_t capacity;       /* C = 2^(32-b), fixed-point mass of one bucket */
  uint32_t id_bytes;       /* 4 if k <= 32 else 8 */
  uint32_t min_len;        /* shortest and longest path length */
  uint32_t max_len;
  uint32_t lds_resident;   /* 1 if generation stages the table in LDS */
  double expected_len;     /* sum_j w_j L_j / 2^32: letters per sample */
  uint64_t export_bytes;   /* bytes written by rmat_table_export */
  uint64_t device_bytes;   /* device memory held by the table */
  uint32_t initiator_k;    /* 2 for R-MAT, K for a K x K Kronecker table */
  uint32_t n_tables;       /* 1, or P for a set of perturbed tables (n_buckets each) */
} rmat_info;

/*
 * Builds the path table (Sec. 2, the priority-queue fragment or the
 * fixed-length strategy) and its alias structure on the current device.
 *
 *  a, b, c, d   quadrant probabilities, each >= 0, |a+b+c+d - 1| <= 1e-9
 *               (Sec. 1).  They are not renormalised.
 *  k            log2 of the node count, 1..64.
 *  table_bound  VARIABLE: 5..2^24, the table gets 1 + 3 ceil((bound-4)/3)
 *               paths (fewer if every path shorter than min(15, k) is
 *               expanded).  FIXED: 4..2^24, l = floor(log4 bound) must be
 *               <= min(15, k).
 *  path_mode    RMAT_FIXED or RMAT_VARIABLE.
 *  out          receives the handle; valid only when RMAT_OK is returned.
 *
 * Tie-breaking of equal probabilities: probability descending, then path
 * length ascending, then the path as base-4 digits (a<b<c<d) ascending; a
 * path's probability is 1.0 multiplied by a (n_a times), then b, c and d,
 * rounding after each product.  Paths of length min(15, k) are never
 * expanded.  Fixed-point weights w_j sum to 2^32 and are p_j * 2^32 rounded
 * by largest remainders (ties to the lower item index).
 *
 * Synchronous: the call returns after the device build finished.  The
 * table is immutable afterwards and may be used from any stream.
 * Errors: RMAT_EINVAL for any invalid argument, RMAT_ENOMEM, RMAT_EDEVICE.
 */
int rmat_build_table(double a, double b, double c, double d, int k,
                     uint64_t table_bound, int path_mode, rmat_table_t* out);

/*
 * rmat_build_table without waiting: validates and sizes on the host (the
 * same errors), allocates the table, enqueues its device build on `stream`
 * (a hipStream_t; NULL = the null stream) and returns.  The build's working
 * arrays belong to the table (device_bytes counts them, about 24 bytes per
 * bucket beside the table's 36), so builds on different streams may overlap.
 * Work on the table is ordered after the build: a generation call on any
 * stream waits for it on the device (no host wait), and rmat_table_info,
 * rmat_table_export and the partitioned calls wait for it on the host.  The
 * table's shape fields are known at once; its length statistics (min_len,
 * max_len, expected_len) once rmat_table_info has waited.  Until the build
 * is known to be finished, a generation draws one counter block per edge in
 * its first pass (the same edges as with two).  A build that fails on the
 * device (RMAT_EINVAL for parameters inside the sum tolerance whose
 * largest-remainder residual is out of range) leaves terminating records;
 * the failure is returned by rmat_table_info and by every later call on the
 * table except rmat_free_table.  rmat_free_table waits for a running build.
 */
int rmat_build_table_async(double a, double b, double c, double d, int k, uint64_t table_bound, int path_mode,
                           void* stream, rmat_table_t* out);

/*
 * Table of a K x K stochastic Kronecker initiator (Sec. 3 generalizations):
 * P holds K^2 probabilities, row-major (cell (i, j) = letter K i + j: row
 * digit i, column digit j), each >= 0, summing to 1 within 1e-9; 2 <= K <= 16;
 * the graph has K^k nodes (K^k <= 2^64) with base-K ids of k digits, the
 * root-most digit most significant.  The table is that of rmat_build_table
 * over the K^2 letters: VARIABLE expands the most probable path while
 * |A| + K^2 - 1 < table_bound (same tie order: probability descending, depth
 * ascending, code ascending, probability = 1.0 times P_x n_x times in letter
 * order), FIXED takes all paths of length floor(log_{K^2} table_bound); no
 * path is longer than min(k, the largest L with K^L <= 2^15).  A sample
 * appends base-K digits: row = row K^take + floor(rowval / K^(L - take)).
 * K = 2 is rmat_build_table(P[0], P[1], P[2], P[3], ...).  For K > 2 the
 * table is built on the device by one workgroup (the boundary path found by
 * bisection over its probability, then the shared weight, alias and record
 * steps), synchronously; rmat_generate and
 * rmat_generate_async work on it (ids uint32 if K^k <= 2^32, else uint64),
 * rmat_table_export exports it (row / col arrays hold digit values), and the
 * epilogue flags, the reduction, partitioned generation and batches reject
 * it (RMAT_EINVAL).  Errors: RMAT_EINVAL, RMAT_ENOMEM, RMAT_EDEVICE.
 */
int rmat_kron_build_table(const double* P, int K, int k, uint64_t table_bound, int path_mode, rmat_table_t* out);

/*
 * A set of P perturbed tables for degree smoothing (Sec. 3, in place of
 * per-step parameter noise): table i is rmat_build_table of (a, b, c, d)
 * with each entry x scaled by 1 + epsilon (2 u - 1) and the four then
 * normalised (divided by their sum), u the 53-bit uniforms (high 53 bits)
 * of SplitMix64 seeded with perturb_seed, drawn table by table in the order
 * a, b, c, d.  Edge e is drawn from table e mod P (exactly the edge
 * rmat_generate would draw from that table alone).  P (n_tables) is a power
 * of two in 1..64; 0 <= epsilon < 1.  All P tables are built in one launch
 * and have the same shape; rmat_table_info reports one member's shape with
 * n_tables = P; rmat_table_export exports member 0 and
 * rmat_table_export_member member i.  rmat_generate(_async),
 * rmat_generate_ex_async and rmat_generate_reduce_async accept the set.
 * With P > 1 each member has at most 2^19 buckets (the set is addressed by
 * 32-bit offsets and a member's offset is a 24-bit product).  Errors: as
 * rmat_build_table; RMAT_EINVAL for n_tables, epsilon or a member table
 * above 2^19 buckets.
 */
int rmat_build_perturbed_table(double a, double b, double c, double d, int k, uint64_t table_bound, int path_mode,
                               int n_tables, double epsilon, uint64_t perturb_seed, rmat_table_t* out);
int rmat_table_export_member(rmat_table_t t, int i, void* host_buf, size_t nbytes);

/* Releases the table's device memory.  NULL is accepted.  The caller must
 * make sure no generation that uses it is still running. */
int rmat_free_table(rmat_table_t t);

/* Fills *out with the table's shape and statistics (host only; waits for an
 * asynchronous build first, and returns its failure). */
int rmat_table_info(rmat_table_t t, rmat_info* out);

/*
 * Copies the table in a canonical host layout, for parity checks: seven
 * arrays of n_buckets entries each, back to back, in this order:
 *   uint64 w[]      fixed-point weights (sum 2^32; 0 for padding)
 *   double p[]      path probabilities (canonical products; 0 for padding)
 *   uint32 len[]    path lengths (0 for padding)
 *   uint32 row[]    row bits of the path, root-most letter most significant
 *   uint32 col[]    column bits
 *   uint32 thr[]    bucket threshold T_i (C for a bucket that aliases itself)
 *   uint32 alias[]  bucket alias A_i (i for a full bucket)
 * nbytes must be at least rmat_info.export_bytes (= 36 * n_buckets).
 * Synchronous.  Errors: RMAT_EINVAL (NULL or short buffer), RMAT_EDEVICE.
 */
int rmat_table_export(rmat_table_t t, void* host_buf, size_t nbytes);

/*
 * Generates edges e = edge_begin .. edge_begin + m - 1 (Sec. 2, the sampling
 * loop; per-edge Philox streams as described above).
 *
 *  seed              64-bit Philox key.
 *  out_src, out_dst  device arrays of m ids each (uint32 if k <= 32, else
 *                    uint64), 4- or 8-byte aligned; slot i holds edge
 *                    edge_begin + i.
 *  stream            hipStream_t to launch on (NULL: the null stream).
 *
 * rmat_generate is synchronous; rmat_generate_async only enqueues.  m = 0 is
 * a no-op.  Errors: RMAT_EINVAL (NULL table or outputs with m > 0),
 * RMAT_ERANGE (edge_begin + m > 2^64), RMAT_EDEVICE (launch failure).
 */
int rmat_generate(rmat_table_t t, uint64_t seed, uint64_t edge_begin,
                  uint64_t m, void* out_src, void* out_dst);
int rmat_generate_async(rmat_table_t t, uint64_t seed, uint64_t edge_begin,
                        uint64_t m, void* out_src, void* out_dst, void* stream);

/*
 * Generalizations of Sec. 3 applied to each edge before it is stored (the
 * same edges as rmat_generate_async otherwise):
 *  RMAT_UNDIRECTED  an undirected graph: an edge in the lower-left triangle
 *                   (src > dst) is mirrored to the upper right, i.e. its ids
 *                   are swapped, so src <= dst for every edge;
 *  RMAT_SCRAMBLE    both ids are relabelled by one bijection pi of [0, 2^k)
 *                   chosen by scramble_key (after the mirror): three rounds
 *                   of x = (x * M_r + C_r) mod 2^k, x ^= x >> ceil(k/2), with
 *                   M_r (odd) and C_r the SplitMix64 outputs of the key in the
 *                   order M_0, C_0, M_1, C_1, M_2, C_2 (M_r with bit 0 set).
 * flags 0 is rmat_generate_async.  Errors as for rmat_generate_async, and
 * RMAT_EINVAL for unknown flags.
 */
enum rmat_generate_flags { RMAT_UNDIRECTED = 1, RMAT_SCRAMBLE = 2 };
int rmat_generate_ex_async(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, int flags,
                           uint64_t scramble_key, void* out_src, void* out_dst, void* stream);

/*
 * Generates the same edges as rmat_generate but stores none of them; instead
 * it reduces them on the device (a consumer that only needs a digest of a
 * huge instance, generated chunk by chunk):
 *  d_hist  device array of 2^hist_bits uint64 counters, incremented by the
 *          histogram of src >> (k - hist_bits)  (hist_bits in 0..min(k, 16));
 *  d_xor   device uint64, XOR-ed with the XOR over the edges of
 *          mix(e, src, dst) = fmix64(e ^ fmix64(src ^ rotl64(dst, 32))),
 *          fmix64 being MurmurHash3's 64-bit finaliser.
 * The caller zeroes both before the first chunk; further chunks accumulate.
 * The edges are generated in sub-chunks of up to 2^28 into a workspace the
 * table owns (2 bytes per edge of a sub-chunk plus 64 MB of per-workgroup
 * counts), allocated by the first call that needs it and freed with the
 * table; reductions on one table must therefore not overlap on the device
 * (issue them on one stream).  Asynchronous on `stream` once the workspace
 * exists.  Errors as for rmat_generate_async, and RMAT_EINVAL for hist_bits
 * out of range.
 */
int rmat_generate_reduce_async(rmat_table_t t, uint64_t seed,
                               uint64_t edge_begin, uint64_t m, int hist_bits,
                               void* d_hist, void* d_xor, void* stream);

/*
 * rmat_generate_reduce_async for callers that cannot allocate device memory
 * (code under stream or graph capture, serving loops, harnesses that forbid
 * hipMalloc): the same arguments and the same results, bit for bit, but the
 * workspace is a fixed array in the library's device data (48 MiB per GPU
 * the library runs on, held until the process ends) instead of one the
 * table allocates.  The edges are reduced in sub-chunks of 2^23 (bins of 2
 * bytes per edge, then the counts of at most 128 workgroups per 2^15-bin
 * window), so no m or hist_bits that rmat_generate_reduce_async accepts is
 * too large.  The call allocates nothing and makes no memset; it only
 * launches kernels on `stream` (the first call on a device also looks up the
 * array's address there).  Every call on one GPU shares that GPU's array:
 * calls that overlap on the device race (issue them on one stream), and
 * only d_hist and d_xor carry results between calls.  Errors as for
 * rmat_generate_reduce_async.
 */
int rmat_generate_reduce_noalloc_async(rmat_table_t t, uint64_t seed,
                                       uint64_t edge_begin, uint64_t m, int hist_bits,
                                       void* d_hist, void* d_xor, void* stream);

/*
 * Out-degrees of the generated graph (the out-degree histogram of a huge
 * instance read literally: one counter per node).  Generates the same edges
 * as rmat_generate, stores none of them, and adds 1 to d_degree[src] for each
 * edge in [edge_begin, edge_begin + m):
 *  d_degree  device array of 2^k uint32 counters (4-byte aligned), owned
 *            and zeroed by the caller; chunks accumulate; a counter wraps
 *            modulo 2^32.
 * R-MAT tables and perturbed sets; a K x K Kronecker table is rejected
 * (RMAT_EINVAL).  No workspace; asynchronous on `stream`; calls on different
 * streams may overlap (the increments are atomic).  Errors as for
 * rmat_generate_async.
 */
int rmat_generate_degrees_async(rmat_table_t t, uint64_t seed, uint64_t edge_begin, uint64_t m, void* d_degree,
                                void* stream);

/*
 * Degree distribution of n_nodes out-degree counters: d_hist[min(d, max_degree)]
 * += 1 for every counter d of d_degree[0 .. n_nodes).
 *  d_degree  device array of n_nodes uint32 (16-byte aligned), read only;
 *  d_hist    device array of max_degree + 1 uint64, zeroed by the caller
 *            (calls accumulate), the last bin counting every degree
 *            >= max_degree.
 * n_nodes <= 2^40, max_degree < 2^31.  Asynchronous on `stream`.  Errors:
 * RMAT_EINVAL (NULL or misaligned pointers, sizes out of range),
 * RMAT_EDEVICE.
 */
int rmat_degree_distribution_async(const void* d_degree, uint64_t n_nodes, uint32_t max_degree, void* d_hist,
                                   void* stream);

/*
 * Partitioned, communication-free generation (Sec. 3): the adjacency matrix
 * is cut into 2^t x 2^t tiles (t = tile_bits, 1 <= t <= min(k - 1, 15)); the
 * m edges (m <= 2^53) are divided over the tiles top-down through the
 * quadrant tree, and a call only visits the subtrees that meet tile rows
 * [row_begin, row_end), so disjoint row ranges can be generated by separate
 * calls (or processes, or GPUs) without communication and together hold
 * exactly m edges.  Each node splits its count n into the four quadrants by
 * n_a = Bin(n, a), n_b = Bin(n - n_a, b / (b+c+d)), n_c = Bin(n - n_a - n_b,
 * c / (c+d)), n_d = the rest (inversion for n min(p, 1-p) < 30, else BTPE
 * [Kachitvichyanukul & Schmeiser 1988]; node (level l, row prefix R, column
 * prefix C) draws 53-bit uniforms from Philox4x32-10 with counter (R, C, i,
 * 2^31 + l)).  Edge j of tile (R, C) samples the remaining k - t letters from
 * the table with counter (j_lo, j_hi, block, 1 + R 2^t + C) and has
 * src = R 2^(k-t) + row, dst = C 2^(k-t) + col.  (A different stream from
 * rmat_generate: same law, different edges.)
 *
 * rmat_partition_counts writes (row_end - row_begin) x 2^t uint64 counts,
 * row-major, to host memory.  rmat_generate_partition writes the edges of
 * those tiles back to back in the same order (tile by tile, j ascending) to
 * out_src / out_dst, which must hold exactly n_out = sum of the counts ids;
 * it is synchronous.  At most 2^18 tiles per call.  Errors: RMAT_EINVAL
 * (arguments, n_out not equal to the edge count), RMAT_ENOMEM, RMAT_EDEVICE.
 */
int rmat_partition_counts(rmat_table_t t, uint64_t seed, uint64_t m, int tile_bits, uint32_t row_begin,
                          uint32_t row_end, uint64_t* counts);
int rmat_generate_partition(rmat_table_t t, uint64_t seed, uint64_t m, int tile_bits, uint32_t row_begin,
                            uint32_t row_end, void* out_src, void* out_dst, uint64_t n_out);

/*
 * As rmat_generate_partition, enqueued on `stream` (a hipStream_t; NULL: the
 * null stream): the call returns once the tile list is copied and the launch
 * enqueued, and the outputs are written when the stream reaches it, so the
 * host can count the next row range meanwhile (Sec. 3: the ranges need no
 * communication).  The table and the outputs must stay alive until then.
 * Each device keeps a ring of four list buffers: a fifth call in flight waits
 * for the oldest launch.  Errors as for rmat_generate_partition.
 */
int rmat_generate_partition_async(rmat_table_t t, uint64_t seed, uint64_t m, int tile_bits, uint32_t row_begin,
                                  uint32_t row_end, void* out_src, void* out_dst, uint64_t n_out, void* stream);

/* ------------------------------------------------------------------------
 * Batches: many independent instances (each its own a..d, k, table, seed,
 * edge range and outputs) built and generated together.  The method is the
 * same per instance (Sec. 2); batching only changes how work reaches the
 * device: one table-build launch for all tables and one persistent
 * generation launch in which workgroups claim runs of 64-edge blocks and
 * restage the LDS table when the instance changes.  Every instance's output
 * equals that of rmat_build_table + rmat_generate with the same arguments.
 * ---------------------------------------------------------------------- */
typedef struct rmat_instance {
  double a, b, c, d;     /* quadrant probabilities, as for rmat_build_table */
  int32_t k;
  int32_t path_mode;     /* RMAT_FIXED or RMAT_VARIABLE */
  uint64_t table_bound;  /* 0: to be chosen by rmat_batch_autotune */
  uint64_t seed;
  uint64_t edge_begin;
  uint64_t m;
  void* out_src;         /* device arrays of m ids (uint32 if k <= 32, else uint64) */
  void* out_dst;
  int32_t flags;         /* RMAT_UNDIRECTED | RMAT_SCRAMBLE, as for rmat_generate_ex_async */
  int32_t reserved;
  uint64_t scramble_key;
} rmat_instance;

typedef struct rmat_batch* rmat_batch_t;

typedef struct rmat_batch_info {
  uint32_t n_instances;
  uint32_t n_launches;    /* generation launches per run (one per id width / table residency) */
  uint32_t n_work_items;  /* runs of blocks claimed by workgroups */
  uint32_t work_blocks;   /* 64-edge blocks per work item */
  uint32_t tile_blocks;   /* blocks per wave tile in the generation kernel (8) */
  uint32_t max_buckets;   /* largest table */
  uint64_t total_edges;
  uint64_t device_bytes;  /* tables, build scratch and work lists held by the batch */
} rmat_batch_info;

typedef struct rmat_autotune_report {
  double search_seconds;     /* wall time of rmat_batch_autotune */
  double calibration_ns;     /* measured device time per (edge x integer op), ns,
                                of 4096-bucket LDS tables */
  uint32_t n_tuned;          /* instances whose table_bound was chosen */
  uint32_t n_candidates;     /* candidate tables built per tuned instance */
  uint32_t work_blocks;      /* measured work-item size for rmat_batch_create */
  uint32_t chosen;           /* 0: the model's bounds; 1: 4096 for all; 2: 8192 for all */
  uint32_t measured;         /* 1 if the choices were timed (outputs given) */
  uint32_t reserved;
  double model_ms;           /* the model's predicted generation time of its bounds */
  double tuned_ms;           /* measured run of the model's bounds (0 if not timed) */
  double all_4096_ms;        /* measured run with bound 4096 (FIXED: 4^6) for all */
  double all_8192_ms;        /* the same with 8192 */
} rmat_autotune_report;

/*
 * Validates every instance (as rmat_build_table and rmat_generate would),
 * sizes and allocates all tables, their build scratch and the work list, and
 * uploads them.  Nothing is built yet.  work_blocks: 64-edge blocks per work
 * item (0: 2048); the work list holds at most 2^28 items (RMAT_EINVAL
 * beyond).  The instance array is copied; outputs must stay valid for
 * every run.  Errors: RMAT_EINVAL (naming the instance), RMAT_ERANGE,
 * RMAT_ENOMEM, RMAT_EDEVICE.
 */
int rmat_batch_create(const rmat_instance* inst, int n, uint32_t work_blocks, rmat_batch_t* out);

/* Enqueues one run on `stream`: all tables are (re)built in one launch, then
 * every instance is generated by persistent launches.  No allocation, memset
 * or host synchronisation, so the call may be captured in a hipGraph. */
int rmat_batch_enqueue(rmat_batch_t b, void* stream);

/* Same run as one hipGraph launch: the first call captures
 * rmat_batch_enqueue into a graph (on a private stream) and instantiates it;
 * every call launches it on `stream`. */
int rmat_batch_launch_graph(rmat_batch_t b, void* stream);

/* Synchronises the device and reports table-build failures of the last run
 * (RMAT_EINVAL / RMAT_EDEVICE naming the instance). */
int rmat_batch_check(rmat_batch_t b);

/* Shape and statistics of instance i's table, as rmat_table_info gives them
 * (synchronous; after a run).  RMAT_EINVAL if the table was not built. */
int rmat_batch_table_info(rmat_batch_t b, int i, rmat_info* out);

/* Table i of the batch in the layout of rmat_table_export (after a run). */
int rmat_batch_table_export(rmat_batch_t b, int i, void* host_buf, size_t nbytes);

int rmat_batch_get_info(rmat_batch_t b, rmat_batch_info* out);

/* Releases the batch (its graph, tables and lists).  NULL is accepted. */
int rmat_batch_free(rmat_batch_t b);

/*
 * Chooses table_bound for every instance whose table_bound is 0 (in place;
 * path_mode is kept), and the work-item size.  Candidates are the powers of
 * two 2^8 .. 2^16 (FIXED: 4^4 .. 4^8, at most 4^min(15,k)): up to 2^13 held
 * in LDS, above that read from L2 (Sec. 4: the table's size and cache
 * residency set the speed).  All candidate tables are
 * built on the device in one launch; each one's path-length law gives the
 * exact expected Philox blocks and samples per edge (Sec. 2: a longer
 * expected path means fewer samples per edge), and the model's cost of an
 * instance is m x (40 x blocks + 11 x samples) integer ops at the measured
 * rate of the candidate's launch class (each LDS table size, whose bytes set
 * how many workgroups a CU holds, and tables read from L2; one-instance
 * batches per class, measured once per process), plus the time to stage an
 * LDS table once per work item.  The LDS tables of a batch run in one launch
 * laid out for the largest, so the model tries each largest LDS size: every
 * instance takes its cheapest candidate no larger (at that size's rate) or
 * read from L2, and the size with the least total wins.  When every tuned
 * instance has its
 * outputs, the model's bounds are then timed on the batch itself against
 * 4096 and against 8192 for all (a single size replaces the model's bounds
 * only if it is faster by more than 1%), and the work-item size (the
 * formula's, a quarter and four times it) timed on that choice; the
 * edges are overwritten by the caller's run.  Without outputs the model
 * decides alone (the same instances get the same bounds on one device).
 * The choice changes the edges (a different table), which is why it is
 * written back.  report may be NULL.  Synchronous.  Errors: RMAT_EINVAL
 * (naming the instance), RMAT_ENOMEM, RMAT_EDEVICE.
 */
int rmat_batch_autotune(rmat_instance* inst, int n, rmat_autotune_report* report);

/* Thread-local description of the last error ("" if none). */
const char* rmat_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RMAT_H */
