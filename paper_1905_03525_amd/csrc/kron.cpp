// kron.cpp -- tables for K x K stochastic Kronecker initiators (Sec. 3).
//
// The letters are the K^2 cells of the initiator, cell (i, j) being letter
// K i + j (row digit i, column digit j); node ids are k-digit base-K numbers.
// The table is the one of Sec. 2 over K^2 letters: the variable-length set
// grows by expanding the most probable path while |A| + K^2 - 1 < bound
// (ties: probability descending, depth ascending, code ascending; a path's
// probability is 1.0 times P_x n_x times for x = 0, 1, ...), or all paths of
// length l = floor(log_{K^2} bound); paths stop at the depth cap, the
// largest L with K^L <= 2^15 (and at most k).  K = 2 is the R-MAT table.
// This file validates and sizes the table and launches its device build
// (kron_table_build_kernel in table_build.hip); the bucket records hold row
// and column digit values instead of bit strings.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rmat.h"
#include "rmat_internal.h"

namespace rmat {
int adopt_table(const rmat_info& info, const double q[4], int kron_K, const TableView& host, void* d_mem,
                double p_second, rmat_table_t* out);
}  // namespace rmat

namespace {

using rmat::set_error;

int depth_cap(int K, int k) {
  int L = 0;
  uint64_t v = 1;
  while (v * static_cast<uint64_t>(K) <= 32768u) {
    v *= static_cast<uint64_t>(K);
    ++L;
  }
  return std::min(L, k);
}

}  // namespace

static int rmat_kron_build_table_body(const double* P, int K, int k, uint64_t table_bound, int path_mode,
                                      rmat_table_t* out) {
  rmat::clear_error();
  if (!out) return set_error(RMAT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!P) return set_error(RMAT_EINVAL, "NULL initiator");
  if (K < 2 || K > 16) return set_error(RMAT_EINVAL, "K %d outside 2..16", K);
  if (K == 2) return rmat_build_table(P[0], P[1], P[2], P[3], k, table_bound, path_mode, out);
  const int letters = K * K;
  double s = 0.0;
  for (int x = 0; x < letters; ++x) {
    if (!(P[x] >= 0.0) || std::isinf(P[x])) return set_error(RMAT_EINVAL, "initiator entry %d is not >= 0", x);
    s += P[x];
  }
  if (std::fabs(s - 1.0) > 1e-9) return set_error(RMAT_EINVAL, "initiator entries sum to %.17g, not 1", s);
  if (k < 1) return set_error(RMAT_EINVAL, "k must be >= 1");
  {
    long double n = 1.0L;  // K^k <= 2^64
    for (int i = 0; i < k; ++i) n *= K;
    if (n > 18446744073709551616.0L) return set_error(RMAT_EINVAL, "K^k exceeds 2^64");
  }
  if (table_bound > rmat::kMaxBound) return set_error(RMAT_EINVAL, "table_bound above 2^24");
  if (path_mode == RMAT_VARIABLE) {
    if (table_bound < static_cast<uint64_t>(letters) + 1)
      return set_error(RMAT_EINVAL, "VARIABLE needs table_bound >= K^2 + 1");
  } else if (path_mode == RMAT_FIXED) {
    if (table_bound < static_cast<uint64_t>(letters)) return set_error(RMAT_EINVAL, "FIXED needs table_bound >= K^2");
  } else {
    return set_error(RMAT_EINVAL, "unknown path mode %d", path_mode);
  }
  int rc = rmat::check_device();
  if (rc) return rc;
  const int cap = depth_cap(K, k);
  const uint64_t L = static_cast<uint64_t>(letters);

  // table shape: t expansions (VARIABLE: while |A| + L - 1 < bound, at most
  // every expandable node), |A| = 1 + t (L - 1); FIXED: all L^l paths
  rmat::Shape S;
  std::memset(&S, 0, sizeof(S));
  S.cap = cap;
  if (path_mode == RMAT_FIXED) {
    int ell = 0;
    uint64_t size = 1;
    while (size * L <= table_bound) {
      size *= L;
      ++ell;
    }
    if (ell > cap) return set_error(RMAT_EINVAL, "FIXED length %d exceeds the depth cap %d", ell, cap);
    S.fixed_len = ell;
    S.n_items = size;
    S.n_expand = (size - 1) / (L - 1);
  } else {
    const uint64_t t = (table_bound - 1 + (L - 2)) / (L - 1) - 1;  // ceil((bound - 1) / (L - 1)) - 1
    uint64_t all_nodes = 0, lp = 1;
    for (int D = 0; D < cap; ++D, lp *= L) all_nodes += lp;
    S.n_expand = std::min(t, all_nodes);
    S.n_items = 1 + S.n_expand * (L - 1);
  }
  int bits = 0;
  while ((1ull << bits) < S.n_items) ++bits;
  S.bucket_bits = bits;
  S.n_buckets = 1ull << bits;
  S.capacity = 1ull << (32 - bits);
  int dbits = 0;
  while ((1u << dbits) < static_cast<uint32_t>(letters)) ++dbits;

  // device memory: the table, then the build's scratch (shared phases'
  // arrays, letter probabilities, packed codes, two search buffers)
  const uint64_t tb = rmat::table_bytes(S);
  const uint64_t common = (rmat::scratch_bytes(S) + 255) / 256 * 256;
  const uint64_t q_bytes = 256 * sizeof(double);
  const uint64_t code_bytes = (S.n_expand * 8 + 255) / 256 * 256;
  const uint64_t bfs_cap = path_mode == RMAT_VARIABLE ? S.n_expand + rmat::kBuildThreads : 0;
  const uint64_t sb = common + q_bytes + code_bytes + 2 * bfs_cap * 8;
  void* d_mem = nullptr;
  void* d_scratch = nullptr;
  hipError_t e = hipMalloc(&d_mem, tb);
  if (e != hipSuccess) return rmat::hip_fail(e, "hipMalloc(kron table)");
  e = hipMalloc(&d_scratch, sb);
  if (e != hipSuccess) {
    (void)hipFree(d_mem);
    return rmat::hip_fail(e, "hipMalloc(kron build scratch)");
  }
  const rmat::TableView V = rmat::place_table(static_cast<char*>(d_mem), S);
  char* scr = static_cast<char*>(d_scratch);
  const double q4[4] = {P[0], P[1], P[2], P[3]};
  rmat::BuildJob job;
  rmat::fill_job(&job, q4, k, path_mode, S, V, scr);
  job.kron_K = K;
  job.letters = letters;
  job.digit_bits = dbits;
  job.qk = reinterpret_cast<const double*>(scr + common);
  job.kcode = reinterpret_cast<uint64_t*>(scr + common + q_bytes);
  job.bfs[0] = reinterpret_cast<uint64_t*>(scr + common + q_bytes + code_bytes);
  job.bfs[1] = job.bfs[0] + bfs_cap;
  job.bfs_cap = bfs_cap;
  rmat::BuildStats st;
  e = hipMemcpy(scr + common, P, static_cast<size_t>(letters) * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = rmat::launch_kron_table_build(job, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e == hipSuccess) e = hipMemcpy(&st, V.stats, sizeof(st), hipMemcpyDeviceToHost);
  (void)hipFree(d_scratch);
  if (e != hipSuccess) {
    (void)hipFree(d_mem);
    return rmat::hip_fail(e, "kron table build");
  }
  if (st.error != 0) {
    (void)hipFree(d_mem);
    return set_error(st.error == rmat::kBuildResidual ? RMAT_EINVAL : RMAT_EDEVICE,
                     "K x K table build failed on the device (code %d)", st.error);
  }
  rmat_info info;
  rmat::fill_info(&info, k, path_mode, table_bound, S, st, tb);
  rc = rmat::adopt_table(info, q4, K, V, d_mem, rmat::p_second_block(st, k), out);
  if (rc) (void)hipFree(d_mem);
  return rc;
}

extern "C" int rmat_kron_build_table(const double* P, int K, int k, uint64_t table_bound, int path_mode,
                                     rmat_table_t* out) {
  RMAT_GUARD("rmat_kron_build_table", rmat_kron_build_table_body(P, K, k, table_bound, path_mode, out));
}
