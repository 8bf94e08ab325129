// rmat_internal.h -- types shared by the host runtime (api.cpp) and the HIP
// kernels of the R-MAT sampler.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <new>

#include "rmat.h"

namespace rmat {

constexpr int kMaxDepthCap = 15;       // longest path: 16-bit fields per id half
constexpr int kBuildThreads = 1024;    // one workgroup builds one table
constexpr int kMaxClasses = 4096;      // letter-count classes of depth < 15: 3060
constexpr uint64_t kMaxBound = 1ull << 24;

// Hot-path bucket record, 16 bytes (one ds_read_b128).  A sample x selects
// bucket i = (x >> 4) mod nb, so its record sits at byte offset
// x & ((nb - 1) << 4) of the table, and keeps the own item when the other
// bits of x, read as f = (x >> (b + 4)) * 16 + (x mod 16), are below T_i:
//   x  thr_abs: T_i spread around the bucket bits, (T_i & ~15) << b | i << 4
//      | (T_i & 15), so that x < thr_abs exactly when f < T_i (the bucket
//      bits of both are i); a full bucket stores i << 4 and an alias equal
//      to itself, so the test never matters
//   y  rows: own item's row value in bits 15..0, the alias item's in 31..16
//   z  cols: the same for the column values
//   w  lens: own length in bits 15..0, the alias's in 31..16
// so each of the three fields the generator needs is one 16-bit half-word
// select.  For 2 x 2 (R-MAT) tables a value holds the path's bits reversed
// (the root-most letter in bit 0), which lets the generator append a path
// with one shift-or at the current fill level; for K x K tables it is the
// base-K number of the path's digits (root-most digit most significant).
struct alignas(16) BucketRecord {
  uint32_t thr_abs, rows, cols, lens;
};

// Device-side results of a table build, read back by the host.
struct BuildStats {
  int32_t error;           // 0 = ok, else an internal error code (see below)
  uint32_t n_items;
  uint32_t min_len, max_len;
  uint64_t sum_wl;         // sum_j w_j * L_j, exact
  uint64_t residual;       // units handed out by largest remainders
  uint64_t len_mass[16];   // sum of w_j over the items of length L (the length law, times 2^32)
};

enum BuildError : int32_t {
  kBuildOk = 0,
  kBuildItemCount = 1,     // leaf count differs from 1 + 3t
  kBuildResidual = 2,      // largest-remainder residual outside [0, n]
  kBuildAlias = 3,         // alias sweep invariant violated
  kBuildClasses = 4,       // more letter-count classes than kMaxClasses
};

// Everything one table build needs; arrays are device memory.
struct BuildJob {
  double q[4];             // a, b, c, d
  int32_t k, mode, cap, bucket_bits;
  int32_t fixed_len;       // FIXED: l; VARIABLE: 0
  uint32_t n_items;        // expected |A|
  uint64_t n_expand;       // t: expanded nodes (VARIABLE), (4^l - 1) / 3 (FIXED)
  uint64_t n_buckets, capacity;
  // outputs (n_buckets entries each)
  BucketRecord* records;
  double* item_p;
  uint64_t* item_w;
  uint32_t *item_len, *item_row, *item_col;
  uint32_t *thr, *alias;
  BuildStats* stats;
  unsigned int* reset_counter;  // if set, zeroed by this build (a batch's work counter)
  // scratch
  uint32_t* lvl_code;      // n_expand entries: expanded nodes, level by level
  uint32_t* lvl_first;     // index of the first expanded child
  uint32_t* lvl_size;      // leaves below the node
  uint32_t* lvl_off;       // tree-order index of the node's first leaf
  uint8_t* lvl_mask;       // which of the 4 children are expanded
  uint32_t* light_idx;     // n_buckets entries each
  uint32_t* heavy_idx;
  uint64_t* light_cum;     // inclusive prefix sums of light deficits C - w
  uint64_t* heavy_cum;     // inclusive prefix sums of heavy excesses w - C
  // K x K Kronecker tables (kron_K > 2; 0 or 2: an R-MAT table): the K^2
  // letter probabilities, the digit width of packed codes (root-most digit
  // most significant), the expanded nodes' codes level by level and two node
  // buffers of bfs_cap codes for the boundary search
  int32_t kron_K, letters, digit_bits, pad_;
  const double* qk;
  uint64_t* kcode;
  uint64_t* bfs[2];
  uint64_t bfs_cap;
};

// Scratch bytes a build needs beyond the table itself.
inline uint64_t build_scratch_bytes(uint64_t n_expand, uint64_t n_buckets) {
  return n_expand * (4 * 4 + 1) + 256 + n_buckets * (4 + 4 + 8 + 8) + 256;
}

// Launchers (defined in the .hip files); return hipSuccess or the launch error.
hipError_t launch_table_build(const BuildJob* d_jobs, int n_jobs, hipStream_t s);
hipError_t launch_table_build_one(const BuildJob& job, hipStream_t s);
// One K x K Kronecker table (job.kron_K > 2), one workgroup.
hipError_t launch_kron_table_build(const BuildJob& job, hipStream_t s);

// One instance of a batched generation (device array).  Block indices are
// relative to first_block = edge_begin >> 6.
struct GenInst {
  const BucketRecord* records;  // table_mask + 1 tables of n_buckets records, back to back
  uint32_t n_buckets;
  uint32_t table_mask;          // edge e reads table e & table_mask (perturbed sets; 0 otherwise)
  uint32_t bmask;               // (n_buckets - 1) << 4: a sample's record offset within its table
  uint32_t k;
  uint32_t key0, key1;
  uint64_t edge_begin, m;
  uint64_t first_block, n_blocks;
  void* out_src;
  void* out_dst;
  // if set (launches with digests enabled), XOR-ed with the XOR over the
  // generated edges of fmix64(e ^ fmix64(src ^ rotl64(dst, 32)))
  unsigned long long* digest;
  uint32_t ctr3;                  // fourth Philox counter word: 0, or 1 + tile id (partitioned generation)
  // 2: the first pass draws counter blocks 0 and 1 of every edge (tables
  // whose edges mostly need more than four samples); otherwise block 0 only
  uint32_t first_blocks = 1;
  uint32_t kron_k;                // K of the K x K initiator (2: R-MAT letters, bit concatenation)
  uint64_t src_prefix, dst_prefix;  // OR-ed into the ids (a tile's row and column offsets)
  // epilogue applied to each edge before it is stored (Sec. 3): bit 0 mirrors
  // an edge with src > dst, bit 1 relabels both ids by the scramble
  uint32_t epi;
  uint32_t scr_shift;             // ceil(k / 2)
  uint64_t scr_mask;              // 2^k - 1
  uint64_t scr_mul[3], scr_add[3];
};

constexpr uint32_t kEpiUndirected = 1, kEpiScramble = 2;

// The scramble's round constants for a key: SplitMix64 outputs in the order
// M0, C0, M1, C1, M2, C2, each M with its lowest bit set; also mask and shift.
void scramble_params(uint64_t key, int k, GenInst* I);

// One SplitMix64 step [Steele, Lea, Flood, OOPSLA'14] (state advanced in place).
uint64_t splitmix64(uint64_t& state);

// A run of 64-edge blocks of one instance; a batch lists them in instance
// order and workgroups claim them through an atomic counter.
struct GenWorkItem {
  uint32_t inst;
  uint32_t n_blocks;
  uint64_t first;        // first block, relative to the instance's first block
  uint32_t n_inst = 1;   // > 1: instances inst .. inst + n_inst - 1, all on one table, each
                         // generated whole by one wave (first and n_blocks unused)
  uint32_t reserved = 0;
};

struct BatchArgs {
  const GenInst* insts;
  const GenWorkItem* items;
  uint32_t n_items;
  unsigned int* counter;   // must be 0 when the launch starts
  uint32_t max_buckets;    // largest table of the batch (LDS staging size)
  int wide;                // k > 32 (64-bit ids)
  int lds;                 // tables staged in LDS
  int digest;              // honour GenInst::digest
  int general;             // some instance has an epilogue or id prefixes
};

hipError_t launch_generate_batch(const BatchArgs& a, hipStream_t s);

// The tiles of a partitioned graph: instances on one table, laid out in list
// order on a line of cost (inst_cost, then its blocks, per instance) that is
// cut into one equal contiguous part per wave of the launch.
struct TilesArgs {
  const GenInst* insts;      // device array of n_inst instances (one table, each with blocks)
  const uint64_t* cum_cost;  // device array of n_inst + 1: sum over the instances before i of
                             // inst_cost + n_blocks
  uint32_t n_inst;
  uint32_t inst_cost;        // an instance's fixed cost, in blocks
  uint64_t total_blocks;     // blocks of all instances
  uint32_t n_buckets;        // the table's buckets (LDS staging size)
  int wide;                  // k > 32 (64-bit ids)
  int lds;                   // table staged in LDS
};

hipError_t launch_generate_tiles(const TilesArgs& a, hipStream_t s);

// Blocks per tile the generation kernels use for a table of this size.
uint32_t tile_blocks(uint32_t table_buckets, int wide, int lds);

// One-time kernel attributes (dynamic LDS above 64 KB).  Not a stream
// operation; call outside any graph capture before the first launch.
hipError_t prepare_kernels();

struct GenerateArgs {
  const BucketRecord* records;
  uint32_t n_buckets;
  int32_t bucket_bits;
  int32_t k;
  uint32_t lds;            // stage the table in LDS
  uint64_t seed;
  uint64_t edge_begin, m;
  void* out_src;
  void* out_dst;
  uint32_t epi;             // kEpiUndirected | kEpiScramble
  uint64_t scramble_key;
  uint32_t kron_k;          // 2: R-MAT bit strings; K > 2: base-K digit values (Kronecker table)
  uint32_t id_bytes;
  uint32_t n_tables;        // perturbed set size (1: a single table)
  uint32_t first_blocks;    // GenInst::first_blocks
  // reduction variant: the edges are generated in sub-chunks of at most
  // bins_cap edges into `bins` (16-bit source prefixes), counted per
  // workgroup into `partials` (reduce_partials_bytes()) and merged into hist
  int32_t hist_bits;
  unsigned long long* hist;
  unsigned long long* xor_out;
  uint16_t* bins;
  uint64_t bins_cap;
  uint32_t* partials;
  uint32_t max_hist_groups; // rows of `partials` per window (0: one per CU)
  // degree variant: counter `degree[src]` incremented once per edge
  uint32_t* degree;
};

// Largest sub-chunk of a reduction (edges) and the workspace it needs.
constexpr uint64_t kReduceChunk = 1ull << 28;
uint64_t reduce_partials_bytes();

// The fixed workspace of the allocation-free reduction: a file-scope device
// array in generate.hip holding the bins of one sub-chunk of
// kStaticReduceChunk edges and the partial counts of kStaticHistGroups
// workgroups.  Fills `a`'s workspace fields with this device's copy; the
// array's address is looked up once per device (hipGetSymbolAddress) on the
// first call with that device current.
constexpr uint64_t kStaticReduceChunk = 1ull << 23;
constexpr uint32_t kStaticHistGroups = 128;
hipError_t static_reduce_workspace(GenerateArgs* a);

hipError_t launch_generate(const GenerateArgs& a, hipStream_t s);
hipError_t launch_generate_degrees(const GenerateArgs& a, hipStream_t s);
// hist[min(degree[i], max_degree)] += 1 for i < n (degree 16-byte aligned).
hipError_t launch_degree_distribution(const uint32_t* degree, uint64_t n, uint32_t max_degree,
                                      unsigned long long* hist, hipStream_t s);
hipError_t launch_generate_reduce(const GenerateArgs& a, hipStream_t s);

// Largest table (in buckets) that generation stages in LDS.
uint32_t lds_table_limit();

// ---- host-side helpers shared by api.cpp and batch.cpp ----------------------

// Shape of a table (step A1): sizes derived from the arguments alone.
struct Shape {
  int cap, fixed_len, bucket_bits;
  uint64_t n_expand, n_items, n_buckets, capacity;
};

// Validates (a, b, c, d, k, bound, mode) and sizes the table; RMAT_OK or
// RMAT_EINVAL with the message set.
int validate_and_size(const double q[4], int k, uint64_t bound, int mode, Shape* s);

// Device pointers of one built table.
struct TableView {
  BucketRecord* records;
  double* p;
  uint64_t* w;
  uint32_t *len, *row, *col, *thr, *alias;
  BuildStats* stats;
};

uint64_t table_bytes(const Shape& S);    // the table itself (kept)
uint64_t scratch_bytes(const Shape& S);  // its build scratch
TableView place_table(char* base, const Shape& S);
void fill_job(BuildJob* job, const double q[4], int k, int mode, const Shape& S, const TableView& V, char* scratch);
int export_table(const TableView& V, uint64_t n_buckets, void* host_buf, size_t nbytes);
// rmat_info of a built table from its shape and device statistics.
void fill_info(rmat_info* I, int k, int path_mode, uint64_t table_bound, const Shape& S, const BuildStats& stats,
               uint64_t device_bytes);
// Clears the calling thread's error message (every entry point starts so).
// Probability that an edge needs more than four samples (four path lengths,
// drawn from the table's length law, sum to fewer than k letters).
double p_second_block(const BuildStats& st, int k);
// Counter blocks the first generation pass draws for every edge: 2 when most
// edges need a second block (the queue of unfinished edges then holds only
// those that need more than eight samples), else 1.
inline uint32_t first_blocks_for(double p_second) { return p_second >= 0.5 ? 2u : 1u; }

void clear_error();
int check_device();
int hip_fail(hipError_t e, const char* what);

// Error reporting shared by every exported function (defined in api.cpp):
// set_error stores the thread-local message and returns `code`;
// check_launch maps hipGetLastError() to RMAT_OK / RMAT_EDEVICE.
int set_error(int code, const char* fmt, ...);
int check_launch(const char* what);

}  // namespace rmat

// The body of an exported function whose host allocations grow with its
// arguments: an exception never crosses the C ABI; a failed host allocation
// is RMAT_ENOMEM, anything else RMAT_EDEVICE.
#define RMAT_GUARD(name, call)                                                      \
  try {                                                                             \
    return call;                                                                    \
  } catch (const std::bad_alloc&) {                                                 \
    return rmat::set_error(RMAT_ENOMEM, "%s: host allocation failed", name);       \
  } catch (...) {                                                                   \
    return rmat::set_error(RMAT_EDEVICE, "%s: unexpected host error", name);      \
  }
